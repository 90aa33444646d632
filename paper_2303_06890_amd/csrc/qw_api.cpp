// Host side of libqw: matrix preprocessing, state management, HIP-graph
// replay of the step loop, the linear solver and the gradient sweep, behind
// the C ABI declared in include/qw.h.
#include "../../include/qw.h"
#include "qw_internal.h"
#include "qw_kappa.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <utility>
#include <vector>

using qw::List;
using qw::Slots;

namespace {

// Last error text of the calling thread (trivially destructible, so the
// library registers nothing to run at thread or process exit).
thread_local char g_err[1024];

int set_err(int code, const std::string& msg) {
  std::snprintf(g_err, sizeof(g_err), "%s", msg.c_str());
  return code;
}
// The same without a std::string (usable where host memory has run out).
int set_err_text(int code, const char* msg) {
  std::snprintf(g_err, sizeof(g_err), "%s", msg);
  return code;
}

// Body of an entry point of the C ABI: no C++ exception leaves the library.
// Host memory exhaustion becomes QW_ENOMEM, anything else QW_EINVAL.
template <class F>
int guarded(F&& f) noexcept {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return set_err_text(QW_ENOMEM, "host memory allocation failed");
  } catch (const std::exception& e) {
    return set_err_text(QW_EINVAL, e.what());
  } catch (...) {
    return set_err_text(QW_EINVAL, "unexpected internal error");
  }
}
// The same for entry points without a status (errors are dropped).
template <class F>
void guarded_void(F&& f) noexcept {
  try {
    f();
  } catch (...) {
  }
}

void prefix_err(const std::string& prefix) {
  const std::string m = prefix + g_err;
  std::snprintf(g_err, sizeof(g_err), "%s", m.c_str());
}

#define QW_HIP(call)                                                                                  \
  do {                                                                                                \
    hipError_t e_ = (call);                                                                           \
    if (e_ != hipSuccess) return set_err(QW_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

int ceil_log2(int64_t x) {
  int r = 0;
  while ((int64_t(1) << r) < x) ++r;
  return r;
}

struct Alloc {
  qw_allocator a{};
  bool custom = false;
  void* get(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    if (custom) return a.alloc(bytes, a.user);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
  }
  // Arrays of 2 MiB and more start on a 2 MiB boundary (`raw` is what put()
  // takes back).  The step kernels' time depends on where the planes fall:
  // moving them off such a boundary cost about 2 % at 16384 x 8 (measured).
  void* get_paged(size_t bytes, void** raw) {
    constexpr uintptr_t kPage = uintptr_t(2) << 20;
    if (bytes < kPage) return *raw = get(bytes);
    char* p = static_cast<char*>(get(bytes + kPage));
    *raw = p;
    if (!p) return nullptr;
    return reinterpret_cast<void*>((reinterpret_cast<uintptr_t>(p) + kPage - 1) & ~(kPage - 1));
  }
  void put(void* p) {
    if (!p) return;
    if (custom)
      a.free(p, a.user);
    else
      (void)hipFree(p);
  }
};

struct HostInst {
  int32_t n = 0, N = 0, nbits = 0, s = 0, hbits = 0;
  double scale = 1.0;
  int64_t item_base = 0, jbase = 0, nnz_base = 0, nnz = 0;
};

}  // namespace

struct qw_ctx {
  // one reference for the caller (dropped by qw_ctx_free) plus one per live
  // state made from this context: the context outlives its states whatever
  // order the caller frees them in
  std::atomic<int> refs{1};
  Alloc alloc;
  // Device buffers of freed states, kept for the next states of this context
  // (one allocation through a caller's allocator can cost several us; a
  // state has eight): at most kPoolPerSize buffers of one size and
  // kPoolBytes in all, released with the context.  A state is freed after a
  // device synchronisation, so no launch still uses a pooled buffer.
  std::mutex pool_mu;
  std::vector<std::pair<size_t, void*>> pool;
  size_t pool_bytes = 0;
  int32_t ninst = 0;
  int32_t nbits = 0;  // key register width
  int64_t items = 0;  // ELL slots incl. alignment padding
  int64_t waves = 0;  // wavefronts of one step-kernel pass
  int64_t jtotal = 0;
  int64_t ntotal = 0;  // sum of unpadded n_i
  int64_t nnz_total = 0;
  std::vector<HostInst> inst;
  std::vector<int64_t> csc_home;  // home of every CSC entry's slot
  // The same on the device (int32: homes < 2^31), and the N-vector index of
  // every unpadded column, for the gradient's gathers into CSC order.
  int32_t* dcsc_home = nullptr;
  int32_t* dcol_row = nullptr;
  // Host copy of the QRAM table (row-major col/val as on the device, the
  // imaginary parts by home), kept for the condition number.
  std::vector<int32_t> hcol;
  std::vector<double> hval;
  std::vector<double> hvim;
  // 1 / min |lambda(A/s)| per instance once computed (NaN before).
  mutable std::mutex kappa_mu;
  std::vector<double> kappa;
  int32_t* col = nullptr;
  double* val = nullptr;
  qw::SlotRec* rec = nullptr;
  uint32_t* slink = nullptr;
  double* sval = nullptr;
  double* sfg = nullptr;     // rotation table (Matrix::sfg): realsym or complex matrices
  void* rec_raw = nullptr;   // allocations behind rec, slink, sval and sfg
  void* slink_raw = nullptr;
  void* sval_raw = nullptr;
  void* sfg_raw = nullptr;
  double* vim = nullptr;          // imaginary parts by home (complex matrices only)
  bool complex_values = false;
  int32_t word = 0;               // fixed-point word length (0: FP64 values)
  // every slot of value 0 has a partner of value 0 or none (see StepArgs::zskip)
  bool zclosed = true;
  // some slot has no partner (its S K(q, 0) branch lives in a Q0 cell; see StepArgs::q0)
  bool q0 = false;
  // a real matrix whose slots of negative value have partners of negative
  // value: from a real b every cell is real or imaginary (see StepArgs::real)
  bool realsym = true;
  qw::Inst* dinst = nullptr;
  int32_t* wave_inst = nullptr;
  qw::Inst inst0{};
  qw::Matrix mat() const {
    qw::Matrix m;
    m.col = col;
    m.val = val;
    m.rec = rec;
    m.slink = slink;
    m.sval = sval;
    m.sfg = sfg;
    m.vim = vim;
    m.inst = dinst;
    m.wave_inst = wave_inst;
    m.items = items;
    m.waves = waves;
    m.rows = jtotal;
    m.ninst = ninst;
    m.nbits = nbits;
    m.smax = smax;
    m.slmax = slmax;
    m.suni = suni;
    m.full = int16_t(full);
    m.angles = word > 0 ? 1 : 0;
    m.wide = wide;
    m.xcd = int16_t(xcd ? -1 : 0);  // the launchers fill in the workgroups per XCD
    m.inst0 = inst0;
    return m;
  }
  int32_t smax = 1;
  int32_t slmax = 1;
  int32_t suni = 0;  // s shared by every instance, else 0
  int32_t full = 0;  // every instance has at least one step-kernel wavefront of rows
  int32_t wide = 0;  // 16 lanes per row for instances with s >= 16 (Matrix::wide)
  int32_t xcd = 0;   // row blocks numbered by XCD in the one-pass kernels (Matrix::xcd)
};

namespace {

struct GraphEntry {
  hipStream_t stream;
  int parity;
  double r1s;  // sign of the R1 storage when the graph starts
  int steps;
  bool real;   // launches of the real-amplitude kernels
  hipGraphExec_t exec;
};

}  // namespace

struct qw_state {
  qw_ctx* ctx = nullptr;
  Slots buf[2]{};           // R0, Q0, Q1 planes of the two parity buffers (R1 unused)
  int cur = 0;              // parity holding the state
  double r1s = 1.0;         // buffer cur^1's Q1 plane holds r1s * (the state's R1)
  List L{};                 // branches without a static home (count on the host)
  unsigned long long* acc = nullptr;  // counts of kept outputs (a Q1 output twice), kMaxWaves entries
  bool counts = true;       // false: the step kernels keep no counts (the solver's private walk)
  // Branches written before the counts were last restarted, and the Q1
  // branches of the state at that point (see total_written).
  int64_t written_base = 0;
  int64_t q1_base = 0;
  // The solver's coefficient window inside a captured graph: kSolverGraphSteps
  // coefficients, then the index of the next replay's first one.
  double* cwin = nullptr;
  double2* b = nullptr;     // device copy of b (N-vector layout)
  double* mbuf = nullptr;   // measurement scratch: max(kMaxGrid, 2*jtotal) doubles
  bool prepared = false;    // created by T~ |b~>
  bool zclean = false;      // R0 and Q0 of the slots of value 0 are 0 (true from T~ |b~> on)
  // Real amplitudes (StepArgs::real): the state may live in 8-byte planes
  // (R0, Q0, Q1 of each parity buffer, allocated on first use) while it is
  // only stepped; every use that changes it otherwise moves it back to the
  // complex planes, and a measurement reads a copy there (complex_copy).
  double* rbuf[2]{};
  bool real_ok = false;     // every amplitude is real (T~ |b~> of a real b)
  bool in_real = false;     // the state is in rbuf
  bool cview = false;       // in_real, and the complex planes hold a copy of it
  int64_t steps_since_init = 0;
  int64_t launches = 0;     // step launches (walk steps and swaps)
  int block = 256;
  int grid = 0;             // 0 = automatic
  std::vector<GraphEntry> graphs;
  std::vector<std::pair<void*, size_t>> owned;  // device buffers and their requested sizes
};

namespace {

// Steps per captured graph of the bulk of a call (even: the parity is kept),
// the most graphs one state keeps, and the length of the solver's graph.
constexpr int kLongGraphSteps = 256;
constexpr int kSingleMax = 32;  // calls (and remainders) of at most this many steps: single launches
constexpr size_t kMaxGraphs = 16;
constexpr int kSolverGraphSteps = 256;  // the solver's graph (and the length of its coefficient window)

// Destroy the state's graphs.  A replay may still be running on any of the
// streams they were made for, and such a stream may since have been
// destroyed by its owner, so the wait is for the whole device, not per stream.
void free_graphs(qw_state* st) {
  if (st->graphs.empty()) return;
  (void)hipDeviceSynchronize();
  for (auto& g : st->graphs) (void)hipGraphExecDestroy(g.exec);
  st->graphs.clear();
}

int step_grid(const qw_state* st) {
  if (st->grid > 0) return st->grid;
  // one pass of the step kernel over the slots and the list
  const int64_t lanes = (st->ctx->waves + (int64_t(st->L.cnt) + qw::kWave - 1) / qw::kWave) * qw::kWave;
  int64_t g = (lanes + st->block - 1) / st->block;
  g = std::max<int64_t>(1, std::min<int64_t>(g, qw::kMaxGrid));
  return int(g);
}

// The state's planes as held in buffer p (the current one for the state
// itself): R1 is buffer p^1's Q1 plane, times r1s.
qw::Slots view(const qw_state* st, int p, double r1s) {
  return qw::Slots{st->buf[p].R0, st->buf[p ^ 1].Q1, st->buf[p].Q0, st->buf[p].Q1, r1s};
}
qw::Slots view(const qw_state* st) { return view(st, st->cur, st->r1s); }

// A walk step leaves the next R1 as -Q1 of the input, the swap as +Q1.
double r1s_after(int mode) { return mode == qw::kStep ? -1.0 : 1.0; }

qw::StepArgs step_args(qw_state* st, int mode, double2* yacc, const double* coef) {
  qw::StepArgs a;
  a.m = st->ctx->mat();
  a.in = view(st);
  a.out = view(st, st->cur ^ 1, r1s_after(mode));
  a.L = st->L;
  a.acc = st->counts ? st->acc : nullptr;
  a.mode = mode;
  a.wpb = 0;  // set by the launcher
  a.tau = qw::kTau;
  a.yacc = yacc;
  a.coef = coef;
  a.zskip = st->ctx->zclosed && st->zclean ? 1 : 0;
  a.real = 0;
  a.q0 = st->ctx->q0 ? 1 : 0;
  return a;
}

// The real planes of buffer p, in the layout of view().
qw::Slots rview(const qw_state* st, int p, double r1s) {
  const int64_t n = st->ctx->items;
  const auto plane = [&](int k, int i) { return reinterpret_cast<double2*>(st->rbuf[k] + i * n); };
  return qw::Slots{plane(p, 0), plane(p ^ 1, 2), plane(p, 1), plane(p, 2), r1s};
}

qw::StepArgs step_args_real(qw_state* st, double2* yacc, const double* coef) {
  qw::StepArgs a = step_args(st, qw::kStep, yacc, coef);
  a.in = rview(st, st->cur, st->r1s);
  a.out = rview(st, st->cur ^ 1, r1s_after(qw::kStep));
  a.real = 1;
  return a;
}

// Whether walk steps (with or without the solver's fused projection) may run
// on one double per cell: a real matrix whose negative values pair up, a
// state from T~ of a real b with an empty list, and the one-pass kernels'
// conditions.
bool real_path(const qw_state* st) {
  const qw_ctx* c = st->ctx;
  return c->realsym && st->real_ok && c->full && st->L.cnt == 0 &&
         int64_t(step_grid(st)) * (st->block / qw::kWave) >= c->waves;
}

void* state_get_paged(qw_state* st, size_t bytes);

// Move the state into the real planes: R0, Q0, Q1 of the current buffer and
// the other buffer's Q1 (the R1 storage); an R0 cell of a slot of negative
// value keeps its imaginary part.  The other buffer's R0 and Q0 are
// outputs of the next step; what that step does not write is 0 in both forms.
int to_real(qw_state* st, hipStream_t stream) {
  if (st->in_real) return QW_OK;
  const int64_t n = st->ctx->items;
  for (int k = 0; k < 2; ++k)
    if (!st->rbuf[k]) {
      st->rbuf[k] = static_cast<double*>(state_get_paged(st, sizeof(double) * 3 * n));
      if (!st->rbuf[k]) return set_err(QW_ENOMEM, "device allocation failed for the real planes");
      QW_HIP(qw::launch_fill(st->rbuf[k], int64_t(sizeof(double)) * 3 * n, stream));
    }
  const double* val = st->ctx->sval;  // R0 cells of slots of negative value are imaginary
  QW_HIP(qw::launch_to_real(st->buf[st->cur].R0, st->rbuf[st->cur], val, n, stream));
  QW_HIP(qw::launch_to_real(st->buf[st->cur].Q0, st->rbuf[st->cur] + n, nullptr, 2 * n, stream));
  QW_HIP(qw::launch_to_real(st->buf[st->cur ^ 1].Q1, st->rbuf[st->cur ^ 1] + 2 * n, nullptr, n, stream));
  st->in_real = true;
  return QW_OK;
}

// A copy of a state on the real planes in the complex planes, for uses that
// only read it (measurements, the export): the state stays on the real
// planes, so the next real walk step needs no conversion back.  The copy
// stands until the real planes change (walk steps, the gradient sweep).
int complex_copy(qw_state* st, hipStream_t stream) {
  if (!st->in_real || st->cview) return QW_OK;
  const int64_t n = st->ctx->items;
  const double* val = st->ctx->sval;
  QW_HIP(qw::launch_to_complex(st->rbuf[st->cur], st->buf[st->cur].R0, val, n, stream));
  QW_HIP(qw::launch_to_complex(st->rbuf[st->cur] + n, st->buf[st->cur].Q0, nullptr, 2 * n, stream));
  QW_HIP(qw::launch_to_complex(st->rbuf[st->cur ^ 1] + 2 * n, st->buf[st->cur ^ 1].Q1, nullptr, n, stream));
  st->cview = true;
  return QW_OK;
}

// And back for good (every use that changes the state other than a real walk
// step calls this first).
int to_complex(qw_state* st, hipStream_t stream) {
  int rc = complex_copy(st, stream);
  if (rc) return rc;
  st->in_real = false;
  st->cview = false;
  return QW_OK;
}

int launch_real(qw_state* st, hipStream_t stream, double2* yacc, const double* coef) {
  qw::StepArgs a = step_args_real(st, yacc, coef);
  QW_HIP(qw::launch_step(a, step_grid(st), st->block, stream));
  st->cur ^= 1;
  st->r1s = r1s_after(qw::kStep);
  ++st->launches;
  return QW_OK;
}

int launch_one(qw_state* st, int mode, hipStream_t stream, double2* yacc = nullptr, const double* coef = nullptr) {
  int rc = to_complex(st, stream);
  if (rc) return rc;
  qw::StepArgs a = step_args(st, mode, yacc, coef);
  QW_HIP(qw::launch_step(a, step_grid(st), st->block, stream));
  st->cur ^= 1;
  st->r1s = r1s_after(mode);
  ++st->launches;
  return QW_OK;
}

// Capture `len` walk steps from the state's present parity and sign into an
// instantiated graph (with the solver's fused projection when yacc is set: a
// window node ahead of the steps copies the replay's coefficients into
// st->cwin, so no step looks its coefficient up through a device-side
// counter).  Capturing runs nothing: the state is left as it was, and each
// replay advances it by `len` steps.
int capture_steps(qw_state* st, int len, hipStream_t stream, bool real, double2* yacc, const double* coefm,
                  hipGraphExec_t* out) {
  int64_t* cbase = reinterpret_cast<int64_t*>(st->cwin + kSolverGraphSteps);
  const int cur0 = st->cur;
  const double r1s0 = st->r1s;
  QW_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int i = 0; i < len && e == hipSuccess; ++i) {
    if (yacc && i == 0) e = qw::launch_coef_window(coefm, cbase, st->cwin, len, -1, stream);
    const double* coef = yacc ? st->cwin + i : nullptr;
    qw::StepArgs a = real ? step_args_real(st, yacc, coef) : step_args(st, qw::kStep, yacc, coef);
    if (e == hipSuccess) e = qw::launch_step(a, step_grid(st), st->block, stream);
    st->cur ^= 1;
    st->r1s = r1s_after(qw::kStep);
  }
  st->cur = cur0;
  st->r1s = r1s0;
  hipGraph_t graph = nullptr;
  const hipError_t ee = hipStreamEndCapture(stream, &graph);
  if (e == hipSuccess) e = ee;
  if (e == hipSuccess) e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return set_err(QW_EDEVICE, std::string("step graph capture: ") + hipGetErrorString(e));
  (void)hipGraphUpload(*out, stream);  // the first replay then starts as fast as the later ones
  return QW_OK;
}

// Replay `reps` times the state's graph of `len` walk steps for its present
// stream, parity, sign and representation, capturing it first if needed.
// A state keeps at most kMaxGraphs graphs (the oldest goes first).
int replay_steps(qw_state* st, int len, int64_t reps, hipStream_t stream, bool real) {
  GraphEntry* ge = nullptr;
  for (auto& g : st->graphs)
    if (g.stream == stream && g.parity == st->cur && g.r1s == st->r1s && g.steps == len && g.real == real) ge = &g;
  if (!ge) {
    if (st->graphs.size() >= kMaxGraphs) {
      // no replay of the evicted graph may still run, on whichever stream it was made for
      QW_HIP(hipDeviceSynchronize());
      (void)hipGraphExecDestroy(st->graphs.front().exec);
      st->graphs.erase(st->graphs.begin());
    }
    hipGraphExec_t exec;
    int rc = capture_steps(st, len, stream, real, nullptr, nullptr, &exec);
    if (rc) return rc;
    st->graphs.push_back({stream, st->cur, st->r1s, len, real, exec});
    ge = &st->graphs.back();
  }
  for (int64_t r = 0; r < reps; ++r) QW_HIP(hipGraphLaunch(ge->exec, stream));
  st->cur ^= int((int64_t(len) * reps) & 1);
  st->r1s = r1s_after(qw::kStep);
  st->launches += reps * len;
  return QW_OK;
}

// Run `n` walk steps.  On a stream, a call of more than kSingleMax steps is
// replayed from captured graphs: as many kLongGraphSteps-step replays as
// fit, then one graph of exactly the remaining count (single launches when
// that is kSingleMax or fewer), each captured on first use and kept with the
// state.  Inside a long graph a kernel follows the previous one about 0.2 us
// sooner than a single launch does, but the start of a replay costs the GPU
// about 10-20 us more than a launch (measured with empty kernels and with
// the step), so short calls are single launches: as fast as a short graph
// when the GPU idles, faster when the launches queue behind other work.  A
// captured graph is replayed back to back, so it starts from the sign a walk
// step leaves: a state fresh from preparation, import or the swap takes its
// first step as a single launch, and so does a state whose long graph exists
// only for the other parity (one launch instead of a second capture).
int run_steps(qw_state* st, int64_t n, hipStream_t stream) {
  if (n == 0) return QW_OK;
  const bool real = real_path(st);
  int rc = real ? to_real(st, stream) : to_complex(st, stream);
  if (rc) return rc;
  st->cview = false;
  const auto one = [&]() {
    --n;
    return real ? launch_real(st, stream, nullptr, nullptr) : launch_one(st, qw::kStep, stream);
  };
  if (stream == nullptr || n <= kSingleMax) {
    while (n > 0)
      if ((rc = one())) return rc;
    return QW_OK;
  }
  const auto have = [&](int len, int parity) {
    for (const auto& g : st->graphs)
      if (g.stream == stream && g.parity == parity && g.r1s == r1s_after(qw::kStep) && g.steps == len &&
          g.real == real)
        return true;
    return false;
  };
  if (n >= 2 && st->r1s != r1s_after(qw::kStep) && (rc = one())) return rc;
  if (n >= kLongGraphSteps) {
    if (n > kLongGraphSteps && !have(kLongGraphSteps, st->cur) && have(kLongGraphSteps, st->cur ^ 1) &&
        (rc = one()))
      return rc;
    const int64_t reps = n / kLongGraphSteps;
    if (reps > 0) {
      if ((rc = replay_steps(st, kLongGraphSteps, reps, stream, real))) return rc;
      n -= reps * kLongGraphSteps;
    }
  }
  if (n > kSingleMax) {
    if ((rc = replay_steps(st, int(n), 1, stream, real))) return rc;
    n = 0;
  }
  while (n > 0)
    if ((rc = one())) return rc;
  return QW_OK;
}

// The solver's walk: `n` steps, the k-th launch of the call adding coefm[k]
// times the projection into yacc; kSolverGraphSteps-step graph replays
// (captured for this call and not kept: y and the table change per solve)
// between single launches.
int run_solver_steps(qw_state* st, int64_t n, hipStream_t stream, double2* yacc, const double* coefm) {
  if (n == 0) return QW_OK;
  const bool real = real_path(st);
  int rc = real ? to_real(st, stream) : to_complex(st, stream);
  if (rc) return rc;
  st->cview = false;
  int64_t k = 0;  // launches of this call so far
  const auto one = [&]() {
    const double* coef = coefm + k;
    ++k;
    --n;
    return real ? launch_real(st, stream, yacc, coef) : launch_one(st, qw::kStep, stream, yacc, coef);
  };
  if (stream != nullptr && n > kSolverGraphSteps) {
    if (st->r1s != r1s_after(qw::kStep) && (rc = one())) return rc;
    const int64_t reps = n / kSolverGraphSteps;
    if (reps > 0) {
      hipGraphExec_t exec;
      if ((rc = capture_steps(st, kSolverGraphSteps, stream, real, yacc, coefm, &exec))) return rc;
      int64_t* cbase = reinterpret_cast<int64_t*>(st->cwin + kSolverGraphSteps);
      hipError_t e = qw::launch_coef_window(coefm, cbase, st->cwin, kSolverGraphSteps, k, stream);
      for (int64_t r = 0; r < reps && e == hipSuccess; ++r) e = hipGraphLaunch(exec, stream);
      const hipError_t es = hipStreamSynchronize(stream);  // before the graph goes
      (void)hipGraphExecDestroy(exec);
      if (e == hipSuccess) e = es;
      if (e != hipSuccess) return set_err(QW_EDEVICE, std::string("solver graph: ") + hipGetErrorString(e));
      st->launches += reps * kSolverGraphSteps;  // even: the parity is kept
      st->r1s = r1s_after(qw::kStep);
      k += reps * kSolverGraphSteps;
      n -= reps * kSolverGraphSteps;
    }
  }
  while (n > 0)
    if ((rc = one())) return rc;
  return QW_OK;
}

// ---- matrix preprocessing ------------------------------------------------------

struct Ell {
  std::vector<int32_t> col;
  std::vector<double> val;
  std::vector<double> vim;  // imaginary parts (complex input only)
};

// Validate one CSC instance, rescale, round s up to a power of two, pad every
// column to s sorted unique slots (filler = smallest absent rows, value 0)
// and the dimension to a power of two.  vals_im: imaginary parts of a
// complex Hermitian matrix, or NULL for a real one.
int preprocess(int32_t n, const int32_t* colptr, const int32_t* rowidx, const double* vals,
               const double* vals_im, double scale_in, uint32_t flags, HostInst& hi, Ell& ell,
               std::vector<int64_t>& slot_of) {
  auto mag = [&](int64_t p) { return vals_im ? std::hypot(vals[p], vals_im[p]) : std::fabs(vals[p]); };
  if (n <= 0) return set_err(QW_EINVAL, "matrix dimension must be positive");
  if (colptr[0] != 0) return set_err(QW_EINVAL, "colptr[0] must be 0");
  int64_t smax = 1;
  double amax = 0.0;
  for (int32_t c = 0; c < n; ++c) {
    if (colptr[c + 1] < colptr[c]) return set_err(QW_EINVAL, "colptr is not monotone");
    smax = std::max<int64_t>(smax, colptr[c + 1] - colptr[c]);
    for (int64_t p = colptr[c]; p < colptr[c + 1]; ++p) {
      if (rowidx[p] < 0 || rowidx[p] >= n) return set_err(QW_EINVAL, "row index out of range");
      if (p > colptr[c] && rowidx[p] <= rowidx[p - 1])
        return set_err(QW_EINVAL, "row indices must be sorted and unique inside a column");
      if (!std::isfinite(vals[p]) || (vals_im && !std::isfinite(vals_im[p])))
        return set_err(QW_EINVAL, "non-finite matrix value");
      amax = std::max(amax, mag(p));
      if (rowidx[p] == c && vals[p] < 0.0)
        return set_err(QW_EINVAL, "negative diagonal entry: not encodable by the walk (<j|T^+ S T|j> = |f|^2/s >= 0)");
      if (rowidx[p] == c && vals_im && vals_im[p] != 0.0)
        return set_err(QW_EINVAL, "diagonal entry with an imaginary part: the matrix is not Hermitian");
    }
  }
  const double scale = scale_in > 0.0 ? scale_in : 1.0 / std::max(1.0, amax);
  if (amax * scale > 1.0) return set_err(QW_EINVAL, "|a| > 1 after scaling");
  if (flags & QW_REQUIRE_SYMMETRIC) {
    for (int32_t c = 0; c < n; ++c)
      for (int64_t p = colptr[c]; p < colptr[c + 1]; ++p) {
        const int32_t r = rowidx[p];
        const int32_t* b = rowidx + colptr[r];
        const int32_t* e = rowidx + colptr[r + 1];
        const int32_t* f = std::lower_bound(b, e, c);
        const int64_t t = colptr[r] + (f - b);  // the mirrored entry (c, r)
        if (f == e || *f != c || vals[t] != vals[p] || (vals_im && vals_im[t] != -vals_im[p]))
          return set_err(QW_EINVAL, vals_im ? "matrix is not Hermitian (pass flags=0 to accept it)"
                                            : "matrix is not symmetric (pass flags=0 to accept it)");
      }
  }
  hi.n = n;
  hi.scale = scale;
  hi.hbits = ceil_log2(smax);
  hi.s = 1 << hi.hbits;
  hi.nbits = std::max(1, ceil_log2(n));
  hi.N = 1 << hi.nbits;
  if (hi.s > qw::kMaxS) return set_err(QW_ENOTSUP, "rows with more than 64 slots are not supported");
  if (hi.s > hi.N) return set_err(QW_EINVAL, "s exceeds the padded dimension");
  ell.col.assign(size_t(hi.N) * hi.s, 0);
  ell.val.assign(size_t(hi.N) * hi.s, 0.0);
  ell.vim.assign(vals_im ? size_t(hi.N) * hi.s : 0, 0.0);
  slot_of.assign(size_t(colptr[n]), -1);
  std::vector<int32_t> rows;
  std::vector<char> present(hi.N, 0);
  for (int32_t c = 0; c < hi.N; ++c) {
    const int64_t p0 = c < n ? colptr[c] : 0, p1 = c < n ? colptr[c + 1] : 0;
    for (int64_t p = p0; p < p1; ++p) present[rowidx[p]] = 1;
    // merge the stored rows with the smallest absent ones
    rows.clear();
    int64_t need = hi.s - (p1 - p0);
    for (int32_t r = 0; need > 0; ++r)
      if (!present[r]) {
        rows.push_back(r);
        --need;
      }
    int64_t p = p0;
    size_t f = 0;
    for (int l = 0; l < hi.s; ++l) {
      const size_t q = size_t(c) * hi.s + l;
      if (p < p1 && (f >= rows.size() || rowidx[p] < rows[f])) {
        ell.col[q] = rowidx[p];
        ell.val[q] = vals[p] * scale;
        if (vals_im) ell.vim[q] = vals_im[p] * scale;
        slot_of[p] = int64_t(q);
        ++p;
      } else {
        ell.col[q] = rows[f++];
        ell.val[q] = 0.0;
      }
    }
    for (int64_t pp = p0; pp < p1; ++pp) present[rowidx[pp]] = 0;
  }
  return QW_OK;
}

// ---- fixed-point data --------------------------------------------------------
// A value a = +-q / 2^w of fixed-point data becomes the signed angle
// y = +-(pi/2 - theta) / pi of its rotation, where theta is the fixed-point
// angle: the square-root register r = floor(sqrt(q 2^w)) (integer square root,
// w fraction bits), the angle register t = the nearest integer to
// arccos(r / 2^w) 2^(w+1) / pi (units of (pi/2) / 2^w), theta = t (pi/2) / 2^w.
// The kernels take f = sin(pi |y|) = cos(theta), g = cos(pi y) = sin(theta);
// y = 0 (f = 0, g = 1) exactly when q = 0.

uint64_t int_sqrt(uint64_t x) {
  uint64_t r = uint64_t(std::sqrt(double(x)));
  while (r > 0 && (unsigned __int128)r * r > x) --r;
  while ((unsigned __int128)(r + 1) * (r + 1) <= x) ++r;
  return r;
}

int fixed_point_angles(int32_t w, std::vector<double>& val) {
  const uint64_t one = uint64_t(1) << w;
  for (double& v : val) {
    const double x = std::fabs(v) * double(one);  // exact (power-of-two scaling)
    if (x != std::floor(x) || x >= double(one))
      return set_err(QW_EINVAL, "value " + std::to_string(v) + " is not a fixed-point number of word length " +
                                    std::to_string(w));
    const uint64_t q = uint64_t(x);
    const uint64_t r = int_sqrt(q << w);
    const uint64_t t =
        uint64_t(std::nearbyint(std::acos(double(r) / double(one)) * (double(uint64_t(1) << (w + 1)) / M_PI)));
    const double y = double(one - t) / double(one << 1);  // exact: t <= 2^w
    v = (v < 0.0 && q != 0) ? -y : y;
  }
  return QW_OK;
}

// Whether every slot of negative value has a partner, also of negative value
// (true of symmetric matrices; see StepArgs::real).
bool negative_slots_paired(const HostInst& hi, const Ell& ell) {
  for (int32_t j = 0; j < hi.N; ++j)
    for (int l = 0; l < hi.s; ++l) {
      const size_t q = size_t(j) * hi.s + l;
      if (!(ell.val[q] < 0.0)) continue;
      const int32_t c = ell.col[q];
      const int32_t* row = ell.col.data() + size_t(c) * hi.s;
      const int32_t* f = std::lower_bound(row, row + hi.s, j);
      if (f == row + hi.s || *f != j || !(ell.val[size_t(c) * hi.s + size_t(f - row)] < 0.0)) return false;
    }
  return true;
}

// Whether every slot (j, l) has a partner: j appears in row col[j, l].
bool every_slot_paired(const HostInst& hi, const Ell& ell) {
  for (int32_t j = 0; j < hi.N; ++j)
    for (int l = 0; l < hi.s; ++l) {
      const int32_t c = ell.col[size_t(j) * hi.s + l];
      const int32_t* row = ell.col.data() + size_t(c) * hi.s;
      const int32_t* f = std::lower_bound(row, row + hi.s, j);
      if (f == row + hi.s || *f != j) return false;
    }
  return true;
}

// Whether every slot of value 0 (a filler, or a stored zero) has a partner of
// value 0 or none.  Then, from T~ |b~> on, the R0 and Q0 cells of these slots
// stay 0: T~ puts b_j f / sqrt(s) = 0 there, and a step moves such a cell only
// to the partner's R0 (negated) or to its own Q0 and back (o0 = (2/s) c f -
// R0 = -R0 for f = 0), so the step kernels may skip them.
bool zero_slots_closed(const HostInst& hi, const Ell& ell) {
  const auto is_zero = [&](size_t q) { return ell.val[q] == 0.0 && (ell.vim.empty() || ell.vim[q] == 0.0); };
  for (int32_t j = 0; j < hi.N; ++j)
    for (int l = 0; l < hi.s; ++l) {
      const size_t q = size_t(j) * hi.s + l;
      if (!is_zero(q)) continue;
      const int32_t c = ell.col[q];
      const int32_t* row = ell.col.data() + size_t(c) * hi.s;
      const int32_t* f = std::lower_bound(row, row + hi.s, j);
      if (f != row + hi.s && *f == j && !is_zero(size_t(c) * hi.s + size_t(f - row))) return false;
    }
  return true;
}

int load_impl(qw_ctx** out, int32_t ninst, const int32_t* n, const int64_t* colptr_off, const int64_t* nnz_off,
              const int32_t* colptr, const int32_t* rowidx, const double* vals, const double* vals_im,
              const double* scales, uint32_t flags, const qw_allocator* alloc, void* stream_v);

// Drop one reference; the last one frees the context's device arrays.
void ctx_release(qw_ctx* ctx) {
  if (ctx->refs.fetch_sub(1) != 1) return;
  (void)hipDeviceSynchronize();
  ctx->alloc.put(ctx->col);
  ctx->alloc.put(ctx->val);
  ctx->alloc.put(ctx->rec_raw);
  ctx->alloc.put(ctx->slink_raw);
  ctx->alloc.put(ctx->sval_raw);
  if (ctx->sfg_raw) ctx->alloc.put(ctx->sfg_raw);
  ctx->alloc.put(ctx->vim);
  ctx->alloc.put(ctx->dinst);
  ctx->alloc.put(ctx->wave_inst);
  ctx->alloc.put(ctx->dcsc_home);
  ctx->alloc.put(ctx->dcol_row);
  for (const auto& e : ctx->pool) ctx->alloc.put(e.second);
  delete ctx;
}

int load_impl(qw_ctx** out, int32_t ninst, const int32_t* n, const int64_t* colptr_off, const int64_t* nnz_off,
              const int32_t* colptr, const int32_t* rowidx, const double* vals, const double* vals_im,
              const double* scales, uint32_t flags, const qw_allocator* alloc, void* stream_v) {
  if (!out) return set_err(QW_EINVAL, "out is NULL");
  *out = nullptr;
  if (ninst <= 0 || !n || !colptr || !rowidx || !vals) return set_err(QW_EINVAL, "missing matrix arrays");
  const int32_t word = int32_t((flags >> 8) & 0x3fu);
  const uint32_t lanes = (flags >> 16) & 0x3u;  // 0: the rule below; 1: 8 lanes per row; 2: 16
  if (lanes == 3) return set_err(QW_EINVAL, "lanes per row: QW_LANES_8 or QW_LANES_16, not both");
  if (word > 32) return set_err(QW_EINVAL, "word length must be 1 ... 32 (0: FP64 values)");
  if (word > 0 && vals_im) return set_err(QW_ENOTSUP, "fixed-point data is provided for real matrices only");
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  qw_ctx* ctx = new qw_ctx;
  if (alloc) {
    if (!alloc->alloc || !alloc->free) {
      delete ctx;
      return set_err(QW_EINVAL, "allocator needs alloc and free");
    }
    ctx->alloc.a = *alloc;
    ctx->alloc.custom = true;
  }
  ctx->ninst = ninst;
  ctx->inst.resize(ninst);
  std::vector<int32_t> hcol;
  std::vector<double> hval;
  std::vector<double> hvim;  // imaginary parts by home (complex input)
  ctx->complex_values = vals_im != nullptr;
  ctx->word = word;
  int64_t items = 0, jbase = 0, nnz_base = 0, ntot = 0;
  int nbits = 1;
  for (int32_t i = 0; i < ninst; ++i) {
    const int64_t co = colptr_off ? colptr_off[i] : 0;
    const int64_t zo = nnz_off ? nnz_off[i] : 0;
    HostInst& hi = ctx->inst[i];
    Ell ell;
    std::vector<int64_t> slot_of;
    int rc = preprocess(n[i], colptr + co, rowidx + zo, vals + zo, vals_im ? vals_im + zo : nullptr,
                        scales ? scales[i] : 0.0, flags, hi, ell, slot_of);
    if (rc == QW_OK && word > 0) rc = fixed_point_angles(word, ell.val);
    if (rc == QW_OK) ctx->zclosed = ctx->zclosed && zero_slots_closed(hi, ell);
    if (rc == QW_OK) ctx->q0 = ctx->q0 || !every_slot_paired(hi, ell);
    if (rc == QW_OK) ctx->realsym = ctx->realsym && !vals_im && negative_slots_paired(hi, ell);
    if (rc) {
      prefix_err("instance " + std::to_string(i) + ": ");
      delete ctx;
      return rc;
    }
    hi.item_base = items;
    hi.jbase = jbase;
    hi.nnz_base = nnz_base;
    hi.nnz = colptr[co + n[i]];
    const int64_t slots = int64_t(hi.N) * hi.s;
    hcol.resize(size_t(items + slots), 0);
    hval.resize(size_t(items + slots), 0.0);
    std::copy(ell.col.begin(), ell.col.end(), hcol.begin() + items);
    std::copy(ell.val.begin(), ell.val.end(), hval.begin() + items);
    if (vals_im) {
      hvim.resize(size_t(items + slots), 0.0);
      for (int64_t q = 0; q < slots; ++q)  // row-major j*s + l -> home l*N + j
        hvim[size_t(items + ((q & (hi.s - 1)) << hi.nbits) + (q >> hi.hbits))] = ell.vim[size_t(q)];
    }
    for (int64_t q : slot_of)  // row-major ELL slot j*s + l -> home l*N + j
      ctx->csc_home.push_back(items + ((q & (hi.s - 1)) << hi.nbits) + (q >> hi.hbits));
    items += (slots + qw::kWave - 1) / qw::kWave * qw::kWave;
    hcol.resize(size_t(items), 0);
    hval.resize(size_t(items), 0.0);
    if (vals_im) hvim.resize(size_t(items), 0.0);
    jbase += hi.N;
    nnz_base += hi.nnz;
    ntot += n[i];
    nbits = std::max(nbits, hi.nbits);
  }
  const int instbits = ceil_log2(ninst);
  if (4 * nbits + 2 + instbits > 64) {
    delete ctx;
    return set_err(QW_ENOTSUP, "register key does not fit 64 bits (4n+2+instance bits > 64)");
  }
  ctx->nbits = nbits;
  ctx->items = items;
  ctx->jtotal = jbase;
  ctx->ntotal = ntot;
  ctx->nnz_total = nnz_base;
  // Step-kernel wavefronts: min(s, 8) lanes share a row and hold s / min(s, 8)
  // slots each, so a wavefront covers 64 / min(s, 8) rows.  A context with
  // at most kWideWaves / 2 wavefronts that way gives instances with s >= 16
  // 16 lanes per row instead (at most twice the wavefronts, half the slots
  // per lane): the shapes of 1024 to 8192 rows with s = 16 or 32 step 7-25 %
  // faster so, while 16384 rows with s = 64 (2048 wavefronts) step slower.
  // The load flags QW_LANES_8 / QW_LANES_16 replace the rule (the autotuner
  // times both).
  int64_t waves8 = 0;
  for (int32_t i = 0; i < ninst; ++i) {
    const int rpw_log = 6 - std::min(ctx->inst[i].hbits, 3);
    waves8 += (int64_t(ctx->inst[i].N) + (int64_t(1) << rpw_log) - 1) >> rpw_log;
  }
  ctx->wide = lanes == 2 ? 1 : lanes == 1 ? 0 : (2 * waves8 <= qw::kWideWaves ? 1 : 0);
  ctx->xcd = (flags & QW_XCD_ROWS) ? 1 : 0;
  std::vector<qw::Inst> dinst(ninst);
  int64_t waves = 0;
  for (int32_t i = 0; i < ninst; ++i) {
    const HostInst& hi = ctx->inst[i];
    const int lpr_log = std::min(hi.hbits, ctx->wide ? 4 : 3);
    const int rpw_log = 6 - lpr_log;
    dinst[i].item_base = hi.item_base;
    dinst[i].jbase = hi.jbase;
    dinst[i].wave_base = waves;
    dinst[i].N = hi.N;
    dinst[i].s = hi.s;
    dinst[i].hbits = hi.hbits;
    dinst[i].nlog = hi.nbits;
    dinst[i].lpr_log = lpr_log;
    dinst[i].sl = hi.s >> lpr_log;
    dinst[i].inv_sqrt_s = 1.0 / std::sqrt(double(hi.s));
    waves += (int64_t(hi.N) + (int64_t(1) << rpw_log) - 1) >> rpw_log;
    ctx->smax = std::max(ctx->smax, hi.s);
    ctx->slmax = std::max(ctx->slmax, dinst[i].sl);
  }
  ctx->waves = waves;
  ctx->inst0 = dinst[0];
  ctx->suni = dinst[0].s;
  ctx->full = 1;
  for (int32_t i = 0; i < ninst; ++i) {
    if (dinst[i].s != ctx->suni) ctx->suni = 0;
    if (dinst[i].N < (64 >> dinst[i].lpr_log)) ctx->full = 0;
  }
  std::vector<int32_t> hwave(static_cast<size_t>(waves));
  for (int32_t i = 0; i < ninst; ++i) {
    const int64_t end = i + 1 < ninst ? dinst[i + 1].wave_base : waves;
    std::fill(hwave.begin() + dinst[i].wave_base, hwave.begin() + end, i);
  }
  ctx->col = static_cast<int32_t*>(ctx->alloc.get(sizeof(int32_t) * items));
  ctx->val = static_cast<double*>(ctx->alloc.get(sizeof(double) * items));
  ctx->rec = static_cast<qw::SlotRec*>(ctx->alloc.get_paged(sizeof(qw::SlotRec) * items, &ctx->rec_raw));
  ctx->slink = static_cast<uint32_t*>(ctx->alloc.get_paged(sizeof(uint32_t) * items, &ctx->slink_raw));
  ctx->sval = static_cast<double*>(ctx->alloc.get_paged(sizeof(double) * items, &ctx->sval_raw));
  const int64_t table_doubles = vals_im ? 4 : (ctx->realsym ? 2 : 0);  // per slot (Matrix::sfg)
  if (table_doubles)
    ctx->sfg = static_cast<double*>(ctx->alloc.get_paged(sizeof(double) * table_doubles * items, &ctx->sfg_raw));
  ctx->dinst = static_cast<qw::Inst*>(ctx->alloc.get(sizeof(qw::Inst) * ninst));
  ctx->wave_inst = static_cast<int32_t*>(ctx->alloc.get(sizeof(int32_t) * waves));
  if (vals_im) ctx->vim = static_cast<double*>(ctx->alloc.get(sizeof(double) * items));
  if (!ctx->col || !ctx->val || !ctx->rec || !ctx->slink || !ctx->sval || !ctx->dinst || !ctx->wave_inst ||
      (vals_im && !ctx->vim) || (table_doubles && !ctx->sfg)) {
    ctx_release(ctx);
    return set_err(QW_ENOMEM, "device allocation failed for the matrix");
  }
  hipError_t e = hipMemcpyAsync(ctx->col, hcol.data(), sizeof(int32_t) * items, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->val, hval.data(), sizeof(double) * items, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->dinst, dinst.data(), sizeof(qw::Inst) * ninst, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && vals_im)
    e = hipMemcpyAsync(ctx->vim, hvim.data(), sizeof(double) * items, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->wave_inst, hwave.data(), sizeof(int32_t) * waves, hipMemcpyHostToDevice, stream);
  std::vector<int32_t> hhome(ctx->csc_home.begin(), ctx->csc_home.end());
  std::vector<int32_t> hrow;
  for (int32_t i = 0; i < ninst; ++i)
    for (int32_t j = 0; j < ctx->inst[i].n; ++j) hrow.push_back(int32_t(ctx->inst[i].jbase + j));
  ctx->dcsc_home = static_cast<int32_t*>(ctx->alloc.get(sizeof(int32_t) * std::max<size_t>(1, hhome.size())));
  ctx->dcol_row = static_cast<int32_t*>(ctx->alloc.get(sizeof(int32_t) * std::max<size_t>(1, hrow.size())));
  if (e == hipSuccess && (!ctx->dcsc_home || !ctx->dcol_row)) e = hipErrorOutOfMemory;
  if (e == hipSuccess && !hhome.empty())
    e = hipMemcpyAsync(ctx->dcsc_home, hhome.data(), sizeof(int32_t) * hhome.size(), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && !hrow.empty())
    e = hipMemcpyAsync(ctx->dcol_row, hrow.data(), sizeof(int32_t) * hrow.size(), hipMemcpyHostToDevice, stream);
  // O_s'^-1 of every reflected output: the QBS of j in row col[q], once per matrix
  if (e == hipSuccess) e = qw::launch_fill(ctx->rec, int64_t(sizeof(qw::SlotRec)) * items, stream);
  if (e == hipSuccess) e = qw::launch_fill(ctx->slink, int64_t(sizeof(uint32_t)) * items, stream);
  if (e == hipSuccess) e = qw::launch_fill(ctx->sval, int64_t(sizeof(double)) * items, stream);
  if (e == hipSuccess) e = qw::launch_qbs_table(ctx->mat(), ctx->rec, ctx->slink, ctx->sval, stream);
  if (e == hipSuccess && ctx->sfg) e = qw::launch_rot_table(ctx->mat(), ctx->sfg, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);  // host vectors go out of scope
  if (e != hipSuccess) {
    ctx_release(ctx);
    return set_err(e == hipErrorOutOfMemory ? QW_ENOMEM : QW_EDEVICE,
                   std::string("matrix upload: ") + hipGetErrorString(e));
  }
  ctx->hcol.swap(hcol);
  ctx->hval.swap(hval);
  ctx->hvim.swap(hvim);
  ctx->kappa.assign(size_t(ninst), std::numeric_limits<double>::quiet_NaN());
  *out = ctx;
  return QW_OK;
}

// 1 / min |lambda(A/s)| of one instance, computed once and kept.
int ctx_kappa(qw_ctx* ctx, int32_t inst, double* out) {
  std::lock_guard<std::mutex> lock(ctx->kappa_mu);
  double& k = ctx->kappa[size_t(inst)];
  if (std::isnan(k)) {
    const HostInst& hi = ctx->inst[size_t(inst)];
    std::string err;
    double lam = 0.0;
    const int rc = qw::min_abs_eigenvalue(hi.n, hi.s, hi.nbits, ctx->hcol.data() + hi.item_base,
                                          ctx->hval.data() + hi.item_base,
                                          ctx->hvim.empty() ? nullptr : ctx->hvim.data() + hi.item_base,
                                          ctx->word > 0, &lam, err);
    if (rc) return set_err(rc, "kappa: " + err);
    k = 1.0 / lam;
  }
  *out = k;
  return QW_OK;
}

// ---- states ---------------------------------------------------------------------

constexpr int kPoolPerSize = 4;
constexpr size_t kPoolBytes = size_t(4) << 30;

// A buffer of `bytes` from the context's pool, else from its allocator.
void* ctx_take(qw_ctx* ctx, size_t bytes) {
  {
    std::lock_guard<std::mutex> lock(ctx->pool_mu);
    for (size_t i = 0; i < ctx->pool.size(); ++i)
      if (ctx->pool[i].first == bytes) {
        void* p = ctx->pool[i].second;
        ctx->pool[i] = ctx->pool.back();
        ctx->pool.pop_back();
        ctx->pool_bytes -= bytes;
        return p;
      }
  }
  return ctx->alloc.get(bytes);
}
// Back to the pool, or to the allocator when the pool is full.
void ctx_give(qw_ctx* ctx, void* p, size_t bytes) {
  {
    std::lock_guard<std::mutex> lock(ctx->pool_mu);
    int same = 0;
    for (const auto& e : ctx->pool) same += e.first == bytes;
    if (same < kPoolPerSize && ctx->pool_bytes + bytes <= kPoolBytes) {
      ctx->pool.push_back({bytes, p});
      ctx->pool_bytes += bytes;
      return;
    }
  }
  ctx->alloc.put(p);
}

void* state_get(qw_state* st, size_t bytes) {
  void* p = ctx_take(st->ctx, bytes);
  if (p) st->owned.push_back({p, bytes});
  return p;
}
// The same, starting on a 2 MiB boundary when 2 MiB or larger.
void* state_get_paged(qw_state* st, size_t bytes) {
  constexpr uintptr_t kPage = uintptr_t(2) << 20;
  if (bytes < kPage) return state_get(st, bytes);
  char* raw = static_cast<char*>(state_get(st, bytes + kPage));
  if (!raw) return nullptr;
  return reinterpret_cast<void*>((reinterpret_cast<uintptr_t>(raw) + kPage - 1) & ~(kPage - 1));
}

// Allocate the general list for `cap` branches (previous contents dropped).
int list_alloc(qw_state* st, uint32_t cap) {
  st->L.cnt = 0;
  if (cap <= st->L.cap) return QW_OK;
  st->L.key = static_cast<uint64_t*>(state_get(st, sizeof(uint64_t) * cap));
  st->L.amp = static_cast<double2*>(state_get(st, sizeof(double2) * cap));
  if (!st->L.key || !st->L.amp) {
    st->L.cap = 0;
    return set_err(QW_ENOMEM, "device allocation failed for the branch list");
  }
  st->L.cap = cap;
  return QW_OK;
}

int state_alloc(qw_ctx* ctx, int64_t list_cap, qw_state** out, hipStream_t stream) {
  if (list_cap < 0 || list_cap > int64_t(0xFFFFFFF0u)) return set_err(QW_EINVAL, "capacity out of range");
  qw_state* st = new qw_state;
  st->ctx = ctx;
  ctx->refs.fetch_add(1);
  const size_t pb = sizeof(double2) * ctx->items;  // one plane
  bool ok = true;
  for (int k = 0; k < 2; ++k) {  // R0, Q0, Q1 per parity buffer
    double2* p = static_cast<double2*>(state_get_paged(st, 3 * pb));
    ok = ok && p;
    st->buf[k] = p ? qw::Slots{p, nullptr, p + ctx->items, p + 2 * ctx->items, 1.0} : qw::Slots{};
  }
  st->acc = static_cast<unsigned long long*>(state_get(st, sizeof(unsigned long long) * qw::kMaxWaves));
  st->cwin = static_cast<double*>(state_get(st, sizeof(double) * (kSolverGraphSteps + 1)));
  st->b = static_cast<double2*>(state_get(st, sizeof(double2) * ctx->jtotal));
  st->mbuf = static_cast<double*>(state_get(st, sizeof(double) * std::max<int64_t>(qw::kMaxGrid, 2 * ctx->jtotal + 2)));
  ok = ok && st->acc && st->cwin && st->b && st->mbuf;
  if (ok && list_cap > 0) ok = list_alloc(st, uint32_t(list_cap)) == QW_OK;
  if (!ok) {
    qw_state_free(st);
    return set_err(QW_ENOMEM, "device allocation failed for the state");
  }
  hipError_t e = hipSuccess;
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = qw::launch_fill(st->buf[k].R0, int64_t(3 * pb), stream);
  if (e == hipSuccess) e = qw::launch_fill(st->acc, sizeof(unsigned long long) * qw::kMaxWaves, stream);
  if (e == hipSuccess) e = qw::launch_fill(st->b, sizeof(double2) * ctx->jtotal, stream);
  if (e != hipSuccess) {
    qw_state_free(st);
    return set_err(QW_EDEVICE, std::string("state clear: ") + hipGetErrorString(e));
  }
  *out = st;
  return QW_OK;
}

// Empty the state: both parities cleared, list emptied.
int state_clear(qw_state* st, hipStream_t stream) {
  const int64_t sb = int64_t(sizeof(double2)) * 3 * st->ctx->items;  // the three planes, contiguous
  for (int k = 0; k < 2; ++k) QW_HIP(qw::launch_fill(st->buf[k].R0, sb, stream));
  st->cur = 0;
  st->r1s = 1.0;
  st->L.cnt = 0;
  return QW_OK;
}

// A state of the 8-byte planes only (the gradient's adjoint state on its
// real path): both parity buffers cleared, no counts, no list.
int state_alloc_real(qw_ctx* ctx, qw_state** out, hipStream_t stream) {
  qw_state* st = new qw_state;
  st->ctx = ctx;
  ctx->refs.fetch_add(1);
  st->counts = false;
  st->real_ok = true;
  st->in_real = true;
  const int64_t bytes = int64_t(sizeof(double)) * 3 * ctx->items;
  for (int k = 0; k < 2; ++k) {
    st->rbuf[k] = static_cast<double*>(state_get_paged(st, size_t(bytes)));
    hipError_t e = st->rbuf[k] ? qw::launch_fill(st->rbuf[k], bytes, stream) : hipErrorOutOfMemory;
    if (e != hipSuccess) {
      qw_state_free(st);
      return set_err(e == hipErrorOutOfMemory ? QW_ENOMEM : QW_EDEVICE, "device allocation failed for the real planes");
    }
  }
  *out = st;
  return QW_OK;
}

// The swap S of a state on the 8-byte planes.
int swap_real(qw_state* st, hipStream_t stream) {
  QW_HIP(qw::launch_swap_real(st->ctx->mat(), rview(st, st->cur, st->r1s), rview(st, st->cur ^ 1, r1s_after(qw::kSwap)),
                              st->counts ? st->acc : nullptr, stream));
  st->cur ^= 1;
  st->r1s = r1s_after(qw::kSwap);
  ++st->launches;
  return QW_OK;
}

// Place unique, validated branches (the state must be empty).
int import_branches(qw_state* st, const std::vector<uint64_t>& keys, const std::vector<double2>& amps,
                    hipStream_t stream) {
  const int64_t m = int64_t(keys.size());
  if (m == 0) return QW_OK;
  qw_ctx* ctx = st->ctx;
  int rc = list_alloc(st, uint32_t(m));
  if (rc) return rc;
  void* dk = ctx->alloc.get(sizeof(uint64_t) * m);
  void* da = ctx->alloc.get(sizeof(double2) * m);
  void* dc = ctx->alloc.get(256);
  uint32_t lcnt = 0;
  hipError_t e = (dk && da && dc) ? hipSuccess : hipErrorOutOfMemory;
  if (e == hipSuccess) e = hipMemcpyAsync(dk, keys.data(), sizeof(uint64_t) * m, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(da, amps.data(), sizeof(double2) * m, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = qw::launch_fill(dc, 256, stream);
  if (e == hipSuccess)
    e = qw::launch_import(ctx->mat(), static_cast<uint64_t*>(dk), static_cast<double2*>(da), m, view(st), st->L,
                          static_cast<uint32_t*>(dc), stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&lcnt, dc, sizeof(uint32_t), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  ctx->alloc.put(dk);
  ctx->alloc.put(da);
  ctx->alloc.put(dc);
  if (e != hipSuccess)
    return set_err(e == hipErrorOutOfMemory ? QW_ENOMEM : QW_EDEVICE, std::string("import: ") + hipGetErrorString(e));
  if (lcnt > st->L.cap) return set_err(QW_ECAPACITY, "branch list overflow during import");
  st->L.cnt = lcnt;
  return QW_OK;
}

// Validate keys against the context's layout; merge equal keys; drop the
// branches at or below the pruning threshold, as every step does (a branch
// stored as R1's source is not pruned again when the next step reads it).
int canonical_branches(const qw_ctx* ctx, const uint64_t* keys, const double* re, const double* im,
                       const double* amps, int64_t m, std::vector<uint64_t>& ok, std::vector<double2>& oa) {
  const int n = ctx->nbits;
  const uint64_t nm = (uint64_t(1) << n) - 1;
  // Keys in strictly increasing order (an exported state) need no sort:
  // they are already unique and in order.
  bool in_order = true;
  for (int64_t t = 1; t < m && in_order; ++t) in_order = keys[t - 1] < keys[t];
  std::vector<int64_t> idx;
  if (!in_order) {
    idx.resize(static_cast<size_t>(m));
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return keys[a] < keys[b]; });
  }
  ok.clear();
  oa.clear();
  ok.reserve(static_cast<size_t>(m));
  oa.reserve(static_cast<size_t>(m));
  for (int64_t t = 0; t < m; ++t) {
    const int64_t i = in_order ? t : idx[size_t(t)];
    const uint64_t key = keys[i];
    const uint64_t inst = key >> (4 * n + 2);
    if (inst >= uint64_t(ctx->ninst)) return set_err(QW_EINVAL, "key with an instance index out of range");
    const HostInst& hi = ctx->inst[inst];
    const uint64_t k = (key >> 1) & nm, kc = (key >> (n + 1)) & nm, j = (key >> (2 * n + 2)) & nm,
                   jc = (key >> (3 * n + 2)) & nm;
    if (k >= uint64_t(hi.N) || j >= uint64_t(hi.N) || kc >= uint64_t(hi.s) || jc >= uint64_t(hi.s))
      return set_err(QW_EINVAL, "key with a register value out of range (j,k < N and j_c,k_c < s required)");
    const double2 a = amps ? make_double2(amps[2 * i], amps[2 * i + 1]) : make_double2(re ? re[i] : 0.0, im ? im[i] : 0.0);
    if (!std::isfinite(a.x) || !std::isfinite(a.y)) return set_err(QW_EINVAL, "non-finite amplitude");
    if (!ok.empty() && ok.back() == key) {
      oa.back().x += a.x;
      oa.back().y += a.y;
    } else {
      ok.push_back(key);
      oa.push_back(a);
    }
  }
  size_t w = 0;
  for (size_t r = 0; r < ok.size(); ++r)
    if (std::fabs(oa[r].x) > qw::kTau || std::fabs(oa[r].y) > qw::kTau) {
      ok[w] = ok[r];
      oa[w] = oa[r];
      ++w;
    }
  ok.resize(w);
  oa.resize(w);
  return QW_OK;
}

int measure_partials(qw_state* st, int kind, double* result, hipStream_t stream) {
  int rc = complex_copy(st, stream);
  if (rc) return rc;
  const int grid = 256;
  QW_HIP(qw::launch_measure(st->ctx->mat(), view(st), st->L, kind, st->mbuf, nullptr, grid, stream));
  std::vector<double> h(grid);
  QW_HIP(hipMemcpyAsync(h.data(), st->mbuf, sizeof(double) * grid, hipMemcpyDeviceToHost, stream));
  QW_HIP(hipStreamSynchronize(stream));
  double t = 0.0;
  for (double v : h) t += v;
  *result = t;
  return QW_OK;
}

// Branches written by all launches so far: the sum over launches of the
// output state's branch count.  A launch counts each kept output once and a
// kept Q1 output twice, the second time for the R1 branch that the next
// launch makes of it without reading it.  Over launches 1..K the counters
// therefore hold the true sum plus (Q1 branches after launch K) minus (Q1
// branches before launch 1).
int total_written(qw_state* st, hipStream_t stream, int64_t* out) {
  // partial sums on the device: 2 KB to copy instead of the whole counter array
  unsigned long long* dsum = reinterpret_cast<unsigned long long*>(st->mbuf);
  unsigned long long part[qw::kSumBlocks];
  QW_HIP(qw::launch_sum_counts(st->acc, qw::kMaxWaves, dsum, stream));
  QW_HIP(hipMemcpyAsync(part, dsum, sizeof(part), hipMemcpyDeviceToHost, stream));
  QW_HIP(hipStreamSynchronize(stream));
  unsigned long long t = 0;
  for (unsigned long long v : part) t += v;
  double q1 = 0.0;
  int rc = measure_partials(st, 4, &q1, stream);
  if (rc) return rc;
  *out = st->written_base + int64_t(t) + st->q1_base - int64_t(std::llround(q1));
  return QW_OK;
}

// Restart the counters after the state was changed by something other than a
// launch of the step kernels (an import); `written` is the total before.
int restart_counts(qw_state* st, int64_t written, hipStream_t stream) {
  QW_HIP(qw::launch_fill(st->acc, sizeof(unsigned long long) * qw::kMaxWaves, stream));
  double q1 = 0.0;
  int rc = measure_partials(st, 4, &q1, stream);
  if (rc) return rc;
  st->written_base = written;
  st->q1_base = int64_t(std::llround(q1));
  return QW_OK;
}

// ---- Chebyshev coefficients (Eq. "fx") --------------------------------------------
// p_i = C(2 beta, beta+i)/4^beta from the central term by the ratio
// p_{i+1} = p_i (beta - i)/(beta + i + 1) in long double; the central term is
// the Wallis product for small beta and the Stirling series of
// ln C(2n, n) - 2n ln 2 otherwise.  a_k = 4 (-1)^k sum_{i > k} p_i.
void cks_coefficients(int64_t beta, int32_t j0, double* out) {
  long double p0;
  if (beta < 64) {
    p0 = 1.0L;
    for (int64_t i = 1; i <= beta; ++i) p0 *= (long double)(2 * i - 1) / (long double)(2 * i);
  } else {
    const long double x = (long double)beta;
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double lp = -0.5L * std::log(pi * x) - 1.0L / (8.0L * x) + 1.0L / (192.0L * x * x * x) -
                           1.0L / (640.0L * x * x * x * x * x) + 17.0L / (14336.0L * x * x * x * x * x * x * x);
    p0 = std::exp(lp);
  }
  const int64_t sd = int64_t(std::sqrt((double)beta / 2.0)) + 1;
  const int64_t imax = std::min<int64_t>(beta, int64_t(j0) + 64 + 40 * sd);
  std::vector<long double> p(size_t(imax) + 2, 0.0L);
  p[0] = p0;
  for (int64_t i = 0; i < imax; ++i) p[i + 1] = p[i] * (long double)(beta - i) / (long double)(beta + i + 1);
  std::vector<long double> suf(size_t(imax) + 2, 0.0L);
  for (int64_t i = imax; i >= 0; --i) suf[i] = suf[i + 1] + p[i];
  for (int32_t k = 0; k <= j0; ++k) {
    const long double tail = (k + 1 <= imax) ? suf[k + 1] : 0.0L;
    out[k] = double(((k & 1) ? -4.0L : 4.0L) * tail);
  }
}

// Argument checks shared by qw_grad, qw_grad_noalloc (real values) and
// qw_grad_complex (complex values).
int grad_check(qw_state* st, const double* w, int32_t nsteps, bool complex_form = false) {
  if (!st || !w) return set_err(QW_EINVAL, "missing argument");
  if (!st->prepared || st->steps_since_init != nsteps)
    return set_err(QW_EINVAL, "qw_grad needs the state made by qw_state_init (T~ start) advanced by exactly nsteps");
  if (st->ctx->complex_values && !complex_form)
    return set_err(QW_ENOTSUP, "a complex Hermitian matrix takes qw_grad_complex");
  if (!st->ctx->complex_values && complex_form) return set_err(QW_ENOTSUP, "a real matrix takes qw_grad");
  if (st->ctx->word > 0)
    return set_err(QW_ENOTSUP, "the gradient is provided for FP64 values only, not fixed-point data");
  return QW_OK;
}

// Device buffers of one gradient sweep: the weights (N-vector layout, padding
// rows 0), dL/dv by home, dL/db, and the results in the caller's order.
struct GradBufs {
  double* dw = nullptr;
  double* dv = nullptr;
  double2* db = nullptr;
  double* dg = nullptr;
  double* dvi = nullptr;  // dL/d(Im v) by home: complex values only (dg then holds nnz more results)
};

// The reverse sweep of the gradient, on the state st (advanced by nsteps from
// T~|b~>) and the adjoint state lam (its planes cleared; on the 8-byte planes
// when `real`, where st is too), with dw holding the weights:
//   Psi_n = S psi_n and Lambda_n = diag(w[k]) Psi_n; nsteps reverse steps
//   (the recomputed state and the adjoint state advance together, dL/dv
//   accumulates); back through S; the gradient through the initial T~;
//   the results gathered into the caller's order and copied out.
// Synchronises the stream; the state is left holding the recomputed T~|b~>.
int grad_sweep(qw_state* st, qw_state* lam, bool real, const GradBufs& gb, int32_t nsteps, double* dvals,
               double* dvals_im, double* db_re, double* db_im, double* loss, hipStream_t stream) {
  qw_ctx* ctx = st->ctx;
  const qw::Matrix mm = ctx->mat();
  double part[256];
  int rc = QW_OK;
  st->cview = false;  // the sweep moves the real planes
  hipError_t e = qw::launch_fill(gb.dv, (sizeof(double) * ctx->items + 15) / 16 * 16, stream);
  if (e == hipSuccess && gb.dvi) e = qw::launch_fill(gb.dvi, (sizeof(double) * ctx->items + 15) / 16 * 16, stream);
  if (e == hipSuccess && real) {
    rc = swap_real(st, stream);
    if (!rc)
      e = qw::launch_weight_real(mm, rview(st, st->cur, st->r1s), rview(lam, lam->cur, lam->r1s), gb.dw, st->mbuf,
                                 256, stream);
  } else if (e == hipSuccess) {
    rc = launch_one(st, qw::kSwap, stream);
    if (!rc) e = qw::launch_weight(mm, view(st), st->L, view(lam), lam->L, gb.dw, st->mbuf, 256, stream);
  }
  // The loss partials stay in st->mbuf (no kernel of the sweep uses it) and
  // come back with the results: a copy to host memory here would hold the
  // host until the GPU got to it, and the sweep's launches behind it.
  for (int32_t t = nsteps; t >= 1 && e == hipSuccess && !rc; --t) {
    qw::AdjArgs a;
    a.m = mm;
    if (real) {
      a.in = rview(st, st->cur, st->r1s);
      a.out = rview(st, st->cur ^ 1, r1s_after(qw::kStep));
      a.lin = rview(lam, lam->cur, lam->r1s);
      a.lout = rview(lam, lam->cur ^ 1, r1s_after(qw::kStep));
    } else {
      a.in = view(st);
      a.out = view(st, st->cur ^ 1, r1s_after(qw::kStep));
      a.lin = view(lam);
      a.lout = view(lam, lam->cur ^ 1, r1s_after(qw::kStep));
    }
    a.L = st->L;
    a.LL = lam->L;
    a.acc = st->counts ? st->acc : nullptr;
    a.lacc = lam->acc;
    a.tau = qw::kTau;
    a.dv = gb.dv;
    a.dvi = gb.dvi;
    a.wpb = 0;  // set by the launcher
    a.real = real ? 1 : 0;
    a.q0 = ctx->q0 ? 1 : 0;
    e = qw::launch_adjoint(a, step_grid(st), st->block, stream);
    st->cur ^= 1;
    lam->cur ^= 1;
    st->r1s = lam->r1s = r1s_after(qw::kStep);
    ++st->launches;
  }
  // back to the unconjugated frame: psi_0 and lambda_0, then the finish
  if (e == hipSuccess && !rc && real) {
    rc = swap_real(st, stream);
    if (!rc) rc = swap_real(lam, stream);
    if (!rc) e = qw::launch_grad_init_real(mm, rview(lam, lam->cur, lam->r1s), st->b, gb.dv, gb.db, stream);
  } else if (e == hipSuccess && !rc) {
    rc = launch_one(st, qw::kSwap, stream);
    if (!rc) rc = launch_one(lam, qw::kSwap, stream);
    if (!rc) e = qw::launch_grad_init(mm, view(lam), st->b, gb.dv, gb.db, gb.dvi, stream);
  }
  // the results in the caller's order (CSC entries; b's columns, real and
  // imaginary parts), gathered on the device and copied straight out
  double* gv = gb.dg;
  double* gbr = gb.dg + ctx->nnz_total;
  double* gbi = gbr + ctx->ntotal;
  double* gvi = gb.dvi ? gbi + ctx->ntotal : nullptr;
  if (e == hipSuccess && !rc)
    e = qw::launch_gather_grad(gb.dv, ctx->dcsc_home, ctx->nnz_total, gb.db, ctx->dcol_row, ctx->ntotal, gv, gbr, gbi,
                               gb.dvi, gvi, stream);
  if (e == hipSuccess && !rc && dvals)
    e = hipMemcpyAsync(dvals, gv, sizeof(double) * ctx->nnz_total, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && !rc && dvals_im && gvi)
    e = hipMemcpyAsync(dvals_im, gvi, sizeof(double) * ctx->nnz_total, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && !rc && db_re)
    e = hipMemcpyAsync(db_re, gbr, sizeof(double) * ctx->ntotal, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && !rc && db_im)
    e = hipMemcpyAsync(db_im, gbi, sizeof(double) * ctx->ntotal, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && !rc) e = hipMemcpyAsync(part, st->mbuf, sizeof(part), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && !rc) e = hipStreamSynchronize(stream);
  (void)hipStreamSynchronize(stream);
  st->steps_since_init = 0;
  if (e != hipSuccess)
    return set_err(e == hipErrorOutOfMemory ? QW_ENOMEM : QW_EDEVICE, std::string("gradient: ") + hipGetErrorString(e));
  if (rc) return rc;
  if (loss) {
    double L = 0.0;
    for (double v : part) L += v;
    *loss = L;
  }
  return QW_OK;
}

}  // namespace

// ================================ C ABI ============================================
extern "C" {

const char* qw_last_error(void) { return g_err; }

int qw_load_csc(qw_ctx** out, int32_t n, const int32_t* colptr, const int32_t* rowidx, const double* vals,
                int64_t nnz, double scale, uint32_t flags, const qw_allocator* alloc, void* stream) {
  return guarded([&]() -> int {
    if (colptr && n > 0 && colptr[n] != nnz) return set_err(QW_EINVAL, "colptr[n] != nnz");
    const int64_t zero = 0;
    return load_impl(out, 1, &n, &zero, &zero, colptr, rowidx, vals, nullptr, scale > 0.0 ? &scale : nullptr, flags,
                     alloc, stream);
  });
}

int qw_load_csc_batched(qw_ctx** out, int32_t ninst, const int32_t* n, const int64_t* colptr_off,
                        const int64_t* nnz_off, const int32_t* colptr, const int32_t* rowidx, const double* vals,
                        const double* scales, uint32_t flags, const qw_allocator* alloc, void* stream) {
  return guarded([&]() -> int {
    if (!colptr_off || !nnz_off) return set_err(QW_EINVAL, "offset arrays are required");
    return load_impl(out, ninst, n, colptr_off, nnz_off, colptr, rowidx, vals, nullptr, scales, flags, alloc, stream);
  });
}

int qw_load_csc_hermitian(qw_ctx** out, int32_t ninst, const int32_t* n, const int64_t* colptr_off,
                          const int64_t* nnz_off, const int32_t* colptr, const int32_t* rowidx, const double* vals_re,
                          const double* vals_im, const double* scales, uint32_t flags, const qw_allocator* alloc,
                          void* stream) {
  return guarded([&]() -> int {
    if (!vals_im) return set_err(QW_EINVAL, "vals_im is required (use qw_load_csc for real matrices)");
    if (ninst > 1 && (!colptr_off || !nnz_off)) return set_err(QW_EINVAL, "offset arrays are required");
    return load_impl(out, ninst, n, colptr_off, nnz_off, colptr, rowidx, vals_re, vals_im, scales, flags, alloc,
                     stream);
  });
}

int32_t qw_ctx_ninst(const qw_ctx* ctx) { return ctx ? ctx->ninst : 0; }

int qw_ctx_info(const qw_ctx* ctx, int32_t inst, int32_t* n_padded, int32_t* s, int32_t* nbits, double* scale,
                double* kappa) {
  return guarded([&]() -> int {
    if (!ctx || inst < 0 || inst >= ctx->ninst) return set_err(QW_EINVAL, "bad context or instance");
    const HostInst& hi = ctx->inst[inst];
    if (n_padded) *n_padded = hi.N;
    if (s) *s = hi.s;
    if (nbits) *nbits = ctx->nbits;
    if (scale) *scale = hi.scale;
    if (kappa) {
      std::lock_guard<std::mutex> lock(ctx->kappa_mu);
      *kappa = ctx->kappa[size_t(inst)];
    }
    return QW_OK;
  });
}

int qw_kappa(qw_ctx* ctx, int32_t inst, double* kappa) {
  return guarded([&]() -> int {
    if (!ctx || inst < 0 || inst >= ctx->ninst || !kappa) return set_err(QW_EINVAL, "bad context, instance or output");
    return ctx_kappa(ctx, inst, kappa);
  });
}

void qw_ctx_free(qw_ctx* ctx) {
  guarded_void([&]() {
    if (ctx) ctx_release(ctx);
  });
}

int qw_state_init(qw_state** out, qw_ctx* ctx, const double* b_re, const double* b_im, uint32_t flags,
                  int64_t capacity, void* stream_v) {
  return guarded([&]() -> int {
    if (!out || !ctx || !b_re) return set_err(QW_EINVAL, "missing argument");
    *out = nullptr;
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    std::vector<double2> hb(static_cast<size_t>(ctx->jtotal), make_double2(0.0, 0.0));
    int64_t src = 0;
    for (int32_t i = 0; i < ctx->ninst; ++i) {
      const HostInst& hi = ctx->inst[i];
      for (int32_t j = 0; j < hi.n; ++j, ++src) {
        const double2 v = make_double2(b_re[src], b_im ? b_im[src] : 0.0);
        if (!std::isfinite(v.x) || !std::isfinite(v.y)) return set_err(QW_EINVAL, "non-finite b");
        hb[size_t(hi.jbase + j)] = v;
      }
    }
    if (capacity < 0) return set_err(QW_EINVAL, "capacity must be >= 0");
    qw_state* st;
    int rc = state_alloc(ctx, capacity, &st, stream);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(st->b, hb.data(), sizeof(double2) * ctx->jtotal, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      qw_state_free(st);
      return set_err(QW_EDEVICE, std::string("b upload: ") + hipGetErrorString(e));
    }
    if (flags & QW_INIT_RAW) {
      std::vector<uint64_t> keys;
      std::vector<double2> amps;
      const int n = ctx->nbits;
      for (int32_t i = 0; i < ctx->ninst; ++i) {
        const HostInst& hi = ctx->inst[i];
        for (int32_t j = 0; j < hi.N; ++j) {
          const double2 v = hb[size_t(hi.jbase + j)];
          if (v.x == 0.0 && v.y == 0.0) continue;
          keys.push_back((uint64_t(i) << (4 * n + 2)) | (uint64_t(j) << (2 * n + 2)));
          amps.push_back(v);
        }
      }
      rc = import_branches(st, keys, amps, stream);
      if (rc == QW_OK) rc = restart_counts(st, 0, stream);
      if (rc) {
        qw_state_free(st);
        return rc;
      }
    } else {
      e = qw::launch_init(ctx->mat(), st->b, view(st), qw::kTau, stream);  // a fresh state: buffer 0, r1s = +1
      if (e != hipSuccess) {
        qw_state_free(st);
        return set_err(QW_EDEVICE, std::string("init: ") + hipGetErrorString(e));
      }
      st->prepared = true;
      st->zclean = true;
      st->real_ok = true;
      if (b_im)
        for (int64_t j = 0; j < ctx->jtotal; ++j) st->real_ok = st->real_ok && hb[size_t(j)].y == 0.0;
    }
    *out = st;
    return QW_OK;
  });
}

void qw_state_free(qw_state* st) {
  guarded_void([&]() {
    if (!st) return;
    (void)hipDeviceSynchronize();
    free_graphs(st);
    qw_ctx* ctx = st->ctx;
    for (const auto& o : st->owned) ctx_give(ctx, o.first, o.second);
    delete st;
    ctx_release(ctx);
  });
}

int qw_set_launch(qw_state* st, int32_t wg_size, int32_t grid) {
  return guarded([&]() -> int {
    if (!st) return set_err(QW_EINVAL, "state is NULL");
    if (wg_size) {
      if (wg_size < 64 || wg_size > 256 || wg_size % 64)
        return set_err(QW_EINVAL, "workgroup size must be 64..256, a multiple of 64");
      st->block = wg_size;
    }
    if (grid) {
      if (grid < 1 || grid > qw::kMaxGrid) return set_err(QW_EINVAL, "grid out of range (1..65536)");
      st->grid = grid;
    }
    free_graphs(st);
    return QW_OK;
  });
}

int qw_step(qw_state* st, int32_t nsteps, void* stream) {
  return guarded([&]() -> int {
    if (!st || nsteps < 0) return set_err(QW_EINVAL, "bad state or step count");
    int rc = run_steps(st, nsteps, static_cast<hipStream_t>(stream));
    if (rc == QW_OK) st->steps_since_init += nsteps;
    return rc;
  });
}

int qw_step_adjoint(qw_state* st, int32_t nsteps, void* stream_v) {
  return guarded([&]() -> int {
    if (!st || nsteps < 0) return set_err(QW_EINVAL, "bad state or step count");
    if (nsteps == 0) return QW_OK;
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    // W^dagger = S W S: swap, walk, swap
    int rc = launch_one(st, qw::kSwap, stream);
    if (!rc) rc = run_steps(st, nsteps, stream);
    if (!rc) rc = launch_one(st, qw::kSwap, stream);
    if (rc == QW_OK) st->steps_since_init -= nsteps;
    return rc;
  });
}

int qw_sync(qw_state* st, void* stream) {
  return guarded([&]() -> int {
    if (!st) return set_err(QW_EINVAL, "state is NULL");
    QW_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    return QW_OK;
  });
}

int qw_measure(qw_state* st, int32_t kind, void* out, int64_t out_len, void* stream_v) {
  return guarded([&]() -> int {
    if (!st || !out) return set_err(QW_EINVAL, "missing argument");
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    qw_ctx* ctx = st->ctx;
    switch (kind) {
      case QW_COUNT: {
        if (out_len < 1) return set_err(QW_EINVAL, "out_len too small");
        double c;
        int rc = measure_partials(st, 0, &c, stream);
        if (!rc) static_cast<int64_t*>(out)[0] = int64_t(std::llround(c));
        return rc;
      }
      case QW_NORM: {
        if (out_len < 1) return set_err(QW_EINVAL, "out_len too small");
        return measure_partials(st, 1, static_cast<double*>(out), stream);
      }
      case QW_J_MARGINAL:
      case QW_PROJECT: {
        const int64_t need = kind == QW_J_MARGINAL ? ctx->jtotal : 2 * ctx->jtotal;
        if (out_len < need) return set_err(QW_EINVAL, "out_len too small");
        int rc = complex_copy(st, stream);
        if (rc) return rc;
        QW_HIP(qw::launch_fill(st->mbuf, (sizeof(double) * need + 15) / 16 * 16, stream));
        QW_HIP(qw::launch_measure(ctx->mat(), view(st), st->L, kind == QW_J_MARGINAL ? 2 : 3, nullptr,
                                  st->mbuf, 256, stream));
        QW_HIP(hipMemcpyAsync(out, st->mbuf, sizeof(double) * need, hipMemcpyDeviceToHost, stream));
        QW_HIP(hipStreamSynchronize(stream));
        return QW_OK;
      }
      case QW_STATS: {
        if (out_len < 5) return set_err(QW_EINVAL, "out_len too small");
        int64_t* o = static_cast<int64_t*>(out);
        double c;
        int rc = measure_partials(st, 0, &c, stream);
        if (rc) return rc;
        int64_t tw;
        rc = total_written(st, stream, &tw);
        if (rc) return rc;
        o[0] = st->launches;
        o[1] = int64_t(std::llround(c));
        o[2] = int64_t(st->L.cap);
        o[3] = int64_t(st->L.cnt);
        o[4] = tw;
        if (out_len >= 6) o[5] = st->real_ok && st->ctx->realsym ? 1 : 0;
        if (out_len >= 7) o[6] = st->ctx->wide ? 16 : 8;
        if (out_len >= 8) o[7] = st->ctx->xcd;
        return QW_OK;
      }
      default:
        return set_err(QW_EINVAL, "unknown measurement kind");
    }
  });
}

namespace {

// qw_export (re, im) and qw_export_complex (amps: re/im interleaved).
int export_sorted(qw_state* st, uint64_t* keys, double* re, double* im, double* amps, int64_t cap, int64_t* m,
                  void* stream_v) {
  return guarded([&]() -> int {
    if (!st || !m) return set_err(QW_EINVAL, "missing argument");
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    int64_t count = 0;
    int rc = qw_measure(st, QW_COUNT, &count, 1, stream_v);
    if (rc) return rc;
    *m = count;
    if (cap < count) return set_err(QW_EINVAL, "output arrays too small: " + std::to_string(count) + " branches");
    if (count == 0) return QW_OK;
    if (!keys) return set_err(QW_EINVAL, "keys is NULL");
    if (count > int64_t(UINT32_MAX))  // the compaction and the sort count in 32 bits
      return set_err(QW_EINVAL, "export of more than 2^32 - 1 branches");
    qw_ctx* ctx = st->ctx;
    // Branches are compacted on the GPU (in no fixed order), then sorted by
    // key there: an LSD radix sort over the 8-bit digit windows that hold a
    // bit on which the keys differ (qwk_key_bits), ping-ponging between two
    // key/amplitude buffers.
    const int64_t tiles = (count + qw::kSortTile - 1) / qw::kSortTile;
    void* dk[2] = {ctx->alloc.get(sizeof(uint64_t) * count), ctx->alloc.get(sizeof(uint64_t) * count)};
    void* da[2] = {ctx->alloc.get(sizeof(double2) * count), ctx->alloc.get(sizeof(double2) * count)};
    void* dh = ctx->alloc.get(sizeof(uint32_t) * 256 * (tiles + 1));
    void* dc = ctx->alloc.get(256);  // the append counter at 0, the key bits at 8 and 16
    struct {
      uint32_t got, pad;
      unsigned long long bits[2];
    } hc = {};
    hipError_t e = (dk[0] && dk[1] && da[0] && da[1] && dh && dc) ? hipSuccess : hipErrorOutOfMemory;
    if (e == hipSuccess) e = qw::launch_fill(dc, 256, stream);
    if (e == hipSuccess)
      e = qw::launch_export(ctx->mat(), view(st), st->L, static_cast<uint64_t*>(dk[0]),
                            static_cast<double2*>(da[0]), static_cast<uint32_t*>(dc), uint32_t(count), stream);
    unsigned long long* dbits = reinterpret_cast<unsigned long long*>(static_cast<char*>(dc) + 8);
    if (e == hipSuccess) e = qw::launch_key_bits(static_cast<uint64_t*>(dk[0]), count, dbits, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&hc, dc, sizeof(hc), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    int cur = 0;
    if (e == hipSuccess && int64_t(hc.got) == count) {
      const unsigned long long differ = hc.bits[0] & hc.bits[1];
      uint32_t* hist = static_cast<uint32_t*>(dh);
      for (int shift = 0; shift < 64 && e == hipSuccess;) {
        if (!((differ >> shift) & 1ull)) {
          ++shift;
          continue;
        }
        e = qw::launch_radix_pass(static_cast<uint64_t*>(dk[cur]), static_cast<double2*>(da[cur]), count, shift,
                                  hist + 256, hist, static_cast<uint64_t*>(dk[1 - cur]),
                                  static_cast<double2*>(da[1 - cur]), stream);
        cur = 1 - cur;
        shift += 8;
      }
      if (e == hipSuccess) e = hipMemcpyAsync(keys, dk[cur], sizeof(uint64_t) * count, hipMemcpyDeviceToHost, stream);
      if (amps) {
        if (e == hipSuccess) e = hipMemcpyAsync(amps, da[cur], sizeof(double2) * count, hipMemcpyDeviceToHost, stream);
      } else if (re || im) {
        // Split into re and im planes in the other buffer, then each goes
        // straight to the caller's array.
        double* dre = static_cast<double*>(da[1 - cur]);
        double* dim = dre + count;
        if (e == hipSuccess) e = qw::launch_split_amps(static_cast<double2*>(da[cur]), count, dre, dim, stream);
        if (e == hipSuccess && re) e = hipMemcpyAsync(re, dre, sizeof(double) * count, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess && im) e = hipMemcpyAsync(im, dim, sizeof(double) * count, hipMemcpyDeviceToHost, stream);
      }
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
    }
    for (void* p : {dk[0], dk[1], da[0], da[1], dh, dc}) ctx->alloc.put(p);
    if (e != hipSuccess)
      return set_err(e == hipErrorOutOfMemory ? QW_ENOMEM : QW_EDEVICE, std::string("export: ") + hipGetErrorString(e));
    if (int64_t(hc.got) != count) return set_err(QW_EDEVICE, "export count mismatch");
    for (int64_t t = 1; t < count; ++t)  // every key is unique: strictly increasing
      if (!(keys[t - 1] < keys[t])) return set_err(QW_EDEVICE, "export: keys out of order");
    return QW_OK;
  });
}

}  // namespace

int qw_export(qw_state* st, uint64_t* keys, double* re, double* im, int64_t cap, int64_t* m, void* stream_v) {
  return export_sorted(st, keys, re, im, nullptr, cap, m, stream_v);
}

int qw_export_complex(qw_state* st, uint64_t* keys, double* amps, int64_t cap, int64_t* m, void* stream_v) {
  return export_sorted(st, keys, nullptr, nullptr, amps, cap, m, stream_v);
}

namespace {

// qw_state_import (re, im) and qw_state_import_complex (amps interleaved).
int import_state(qw_state* st, const uint64_t* keys, const double* re, const double* im, const double* amps,
                 int64_t m, void* stream_v) {
  return guarded([&]() -> int {
    if (!st || m < 0 || (m > 0 && (!keys || (!re && !amps)))) return set_err(QW_EINVAL, "missing argument");
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    std::vector<uint64_t> k;
    std::vector<double2> a;
    int rc = canonical_branches(st->ctx, keys, re, im, amps, m, k, a);
    if (rc) return rc;
    int64_t written = 0;
    rc = total_written(st, stream, &written);
    if (rc) return rc;
    rc = state_clear(st, stream);
    if (rc) return rc;
    st->prepared = false;
    st->zclean = false;  // imported branches may sit in R0 or Q0 of slots of value 0
    st->real_ok = false;
    st->in_real = false;  // state_clear empties the complex planes, which hold the state from here
    st->cview = false;
    st->steps_since_init = 0;
    free_graphs(st);  // the list pointers and the kernel arguments change
    rc = import_branches(st, k, a, stream);
    if (rc) return rc;
    return restart_counts(st, written, stream);
  });
}

}  // namespace

int qw_state_import(qw_state* st, const uint64_t* keys, const double* re, const double* im, int64_t m,
                    void* stream_v) {
  return import_state(st, keys, re, im, nullptr, m, stream_v);
}

int qw_state_import_complex(qw_state* st, const uint64_t* keys, const double* amps, int64_t m, void* stream_v) {
  return import_state(st, keys, nullptr, nullptr, amps, m, stream_v);
}

int qw_cks_coeffs(int64_t beta, int32_t j0, double* out) {
  return guarded([&]() -> int {
    if (beta < 1 || j0 < 0 || !out) return set_err(QW_EINVAL, "bad arguments");
    cks_coefficients(beta, j0, out);
    return QW_OK;
  });
}

int qls_run(qw_ctx* ctx, const double* b, double kappa, double eps, int32_t j0_override, double* x_re,
            double* x_im, double* y_norm, double* p_succ, int64_t* walk_steps, void* stream_v) {
  return guarded([&]() -> int {
    if (!ctx || !b) return set_err(QW_EINVAL, "missing argument");
    if (!(eps > 0.0 && eps < 1.0)) return set_err(QW_EINVAL, "eps must lie in (0, 1)");
    if (kappa <= 0.0) {  // the library's own condition number of A/s
      int rck = ctx_kappa(ctx, 0, &kappa);
      if (rck) return rck;
      if (!(kappa >= 1.0)) return set_err(QW_EINVAL, "computed kappa below 1");
    } else if (!(kappa > 1.0) || !std::isfinite(kappa)) {
      return set_err(QW_EINVAL, "kappa must be > 1 (or <= 0 for the library's own)");
    }
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    const double bb = std::ceil(kappa * kappa * std::log(kappa / eps));
    const double j0d = std::ceil(std::sqrt(bb * std::log(4.0 * bb / eps)));
    if (!(bb < 1e15) || !(j0d < 1e9))
      return set_err(QW_EINVAL, "kappa " + std::to_string(kappa) + " needs a schedule of more than 2e9 walk steps");
    const int64_t beta = int64_t(bb);
    int32_t j0 = int32_t(j0d);
    if (j0_override >= 0) j0 = j0_override;
    std::vector<double> a(static_cast<size_t>(j0) + 1);
    cks_coefficients(beta, j0, a.data());
    const int64_t nsteps = 2 * int64_t(j0) + 1;
    // coefficient per input step number m: a_{(m-1)/2} for odd m
    std::vector<double> coefm(static_cast<size_t>(nsteps) + 1, 0.0);
    for (int64_t mm = 1; mm <= nsteps; mm += 2) coefm[size_t(mm)] = a[size_t((mm - 1) / 2)];
    // the solver works on instance 0 only
    std::vector<double> bfull(static_cast<size_t>(ctx->ntotal), 0.0);
    for (int32_t j = 0; j < ctx->inst[0].n; ++j) bfull[size_t(j)] = b[j];
    // host buffers first: nothing below may throw while device resources are held
    std::vector<double2> hy(static_cast<size_t>(ctx->jtotal));
    std::vector<double> proj(2 * static_cast<size_t>(ctx->jtotal));
    qw_state* st = nullptr;
    int rc = qw_state_init(&st, ctx, bfull.data(), nullptr, 0, 0, stream_v);
    if (rc) return rc;
    st->counts = false;  // nobody reads this walk's branch counts
    const int64_t N = ctx->inst[0].N;
    double* dcoef = static_cast<double*>(ctx->alloc.get(sizeof(double) * coefm.size()));
    double2* y = static_cast<double2*>(ctx->alloc.get(sizeof(double2) * ctx->jtotal));
    hipError_t e = (dcoef && y) ? hipSuccess : hipErrorOutOfMemory;
    if (e == hipSuccess)
      e = hipMemcpyAsync(dcoef, coefm.data(), sizeof(double) * coefm.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = qw::launch_fill(y, sizeof(double2) * ctx->jtotal, stream);
    if (e == hipSuccess) {
      rc = run_solver_steps(st, nsteps, stream, y, dcoef);
      if (!rc) rc = qw_measure(st, QW_PROJECT, proj.data(), int64_t(proj.size()), stream_v);
      if (!rc) {
        e = hipMemcpyAsync(hy.data(), y, sizeof(double2) * ctx->jtotal, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
      }
    }
    ctx->alloc.put(dcoef);
    ctx->alloc.put(y);
    qw_state_free(st);
    if (e != hipSuccess) return set_err(e == hipErrorOutOfMemory ? QW_ENOMEM : QW_EDEVICE, "linear solver failed");
    if (rc) return rc;
    // y = sum_k a_k tau_k; the post-selected state is y / |y| (the success
    // probability of the LCU is |y|^2 / (sum_k |a_k|)^2)
    double norm2 = 0.0, asum = 0.0;
    for (double v : a) asum += std::fabs(v);
    for (int64_t j = 0; j < N; ++j) {
      hy[size_t(j)].x += a[size_t(j0)] * proj[2 * size_t(j)];
      hy[size_t(j)].y += a[size_t(j0)] * proj[2 * size_t(j) + 1];
      norm2 += hy[size_t(j)].x * hy[size_t(j)].x + hy[size_t(j)].y * hy[size_t(j)].y;
    }
    const double yn = std::sqrt(norm2);
    if (!(yn > 0.0)) return set_err(QW_EINVAL, "the solver's output vanishes (b = 0?)");
    for (int32_t j = 0; j < ctx->inst[0].n; ++j) {
      if (x_re) x_re[j] = hy[size_t(j)].x / yn;
      if (x_im) x_im[j] = hy[size_t(j)].y / yn;
    }
    if (y_norm) *y_norm = yn;
    if (p_succ) *p_succ = norm2 / (asum * asum);
    if (walk_steps) *walk_steps = nsteps;
    return QW_OK;
  });
}

}  // extern "C"

namespace {

// qw_grad and qw_grad_complex: the sweep on buffers of the context's pool;
// dvals_im is used for complex values only.
int grad_impl(qw_state* st, const double* w, int32_t nsteps, double* dvals, double* dvals_im, double* db_re,
              double* db_im, double* loss, void* stream_v, bool complex_form) {
  return guarded([&]() -> int {
    int rc = grad_check(st, w, nsteps, complex_form);
    if (rc) return rc;
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    const bool real = !complex_form && real_path(st);
    rc = real ? to_real(st, stream) : to_complex(st, stream);
    if (rc) return rc;
    qw_ctx* ctx = st->ctx;
    std::vector<double> hw(static_cast<size_t>(ctx->jtotal), 0.0);
    int64_t src = 0;
    for (int32_t i = 0; i < ctx->ninst; ++i)
      for (int32_t j = 0; j < ctx->inst[i].n; ++j, ++src) hw[size_t(ctx->inst[i].jbase + j)] = w[src];
    qw_state* lam = nullptr;
    rc = real ? state_alloc_real(ctx, &lam, stream) : state_alloc(ctx, st->L.cap, &lam, stream);
    if (rc) return rc;
    lam->L.cnt = st->L.cnt;
    GradBufs gb;
    gb.dw = static_cast<double*>(ctx_take(ctx, sizeof(double) * ctx->jtotal));
    gb.dv = static_cast<double*>(ctx_take(ctx, sizeof(double) * ctx->items));
    gb.db = static_cast<double2*>(ctx_take(ctx, sizeof(double2) * ctx->jtotal));
    const size_t gbytes = sizeof(double) * size_t((complex_form ? 2 : 1) * ctx->nnz_total + 2 * ctx->ntotal);
    gb.dg = static_cast<double*>(ctx_take(ctx, gbytes));
    if (complex_form) gb.dvi = static_cast<double*>(ctx_take(ctx, sizeof(double) * ctx->items));
    hipError_t e = (gb.dw && gb.dv && gb.db && gb.dg && (gb.dvi || !complex_form)) ? hipSuccess : hipErrorOutOfMemory;
    if (e == hipSuccess)
      e = hipMemcpyAsync(gb.dw, hw.data(), sizeof(double) * ctx->jtotal, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
      rc = grad_sweep(st, lam, real, gb, nsteps, dvals, dvals_im, db_re, db_im, loss, stream);
    (void)hipStreamSynchronize(stream);  // after an error too: nothing may still use the buffers
    if (gb.dw) ctx_give(ctx, gb.dw, sizeof(double) * ctx->jtotal);
    if (gb.dv) ctx_give(ctx, gb.dv, sizeof(double) * ctx->items);
    if (gb.db) ctx_give(ctx, gb.db, sizeof(double2) * ctx->jtotal);
    if (gb.dg) ctx_give(ctx, gb.dg, gbytes);
    if (gb.dvi) ctx_give(ctx, gb.dvi, sizeof(double) * ctx->items);
    qw_state_free(lam);
    if (e != hipSuccess)
      return set_err(e == hipErrorOutOfMemory ? QW_ENOMEM : QW_EDEVICE, std::string("gradient: ") + hipGetErrorString(e));
    return rc;
  });
}

}  // namespace

extern "C" {

int qw_grad(qw_state* st, const double* w, int32_t nsteps, double* dvals, double* db_re, double* db_im,
            double* loss, void* stream) {
  return grad_impl(st, w, nsteps, dvals, nullptr, db_re, db_im, loss, stream, false);
}

int qw_grad_complex(qw_state* st, const double* w, int32_t nsteps, double* dvals_re, double* dvals_im,
                    double* db_re, double* db_im, double* loss, void* stream) {
  return grad_impl(st, w, nsteps, dvals_re, dvals_im, db_re, db_im, loss, stream, true);
}

int qw_grad_noalloc(qw_state* st, const double* w, int32_t nsteps, double* dvals, double* db_re, double* db_im,
                    double* loss, void* stream_v) {
  return guarded([&]() -> int {
    int rc = grad_check(st, w, nsteps);
    if (rc) return rc;
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    qw_ctx* ctx = st->ctx;
    if (!real_path(st) || !st->rbuf[0] || !st->rbuf[1])
      return set_err(QW_ENOTSUP,
                     "qw_grad_noalloc needs a state whose walk steps run on one double per cell and have run "
                     "(a real symmetric matrix, a real b, one-pass launch shape, at least one step); use qw_grad");
    // the library's device array: the adjoint state's two parity buffers of
    // three 8-byte planes, the weights, dL/dv by home, dL/db, and the results
    // in the caller's order, each on a 256-byte boundary
    const auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t planes = up(sizeof(double) * 3 * size_t(ctx->items));
    const size_t need = 2 * planes + up(sizeof(double) * size_t(ctx->jtotal)) + up(sizeof(double) * size_t(ctx->items)) +
                        up(sizeof(double2) * size_t(ctx->jtotal)) +
                        up(sizeof(double) * size_t(ctx->nnz_total + 2 * ctx->ntotal));
    void* base = nullptr;
    size_t have = 0;
    QW_HIP(qw::device_scratch(&base, &have));
    if (need > have) {
      char msg[256];
      std::snprintf(msg, sizeof(msg),
                    "qw_grad_noalloc: this context needs %zu bytes of the library's device array, which holds %zu "
                    "(%lld slots); use qw_grad",
                    need, have, static_cast<long long>(ctx->items));
      return set_err_text(QW_EINVAL, msg);
    }
    char* p = static_cast<char*>(base);
    const auto carve = [&](size_t bytes) {
      char* q = p;
      p += up(bytes);
      return q;
    };
    // the adjoint state: a qw_state on the stack over two buffers of the
    // array (its vectors stay empty; it holds no reference on the context
    // and is never freed)
    qw_state lam;
    lam.ctx = ctx;
    lam.counts = false;
    lam.real_ok = true;
    lam.in_real = true;
    lam.rbuf[0] = reinterpret_cast<double*>(carve(planes));
    lam.rbuf[1] = reinterpret_cast<double*>(carve(planes));
    GradBufs gb;
    gb.dw = reinterpret_cast<double*>(carve(sizeof(double) * size_t(ctx->jtotal)));
    gb.dv = reinterpret_cast<double*>(carve(sizeof(double) * size_t(ctx->items)));
    gb.db = reinterpret_cast<double2*>(carve(sizeof(double2) * size_t(ctx->jtotal)));
    gb.dg = reinterpret_cast<double*>(carve(sizeof(double) * size_t(ctx->nnz_total + 2 * ctx->ntotal)));
    rc = to_real(st, stream);  // the state's own 8-byte planes exist (checked above): a conversion at most
    if (rc) return rc;
    // the array keeps the last call's contents: clear what must start at 0
    // (a fill kernel, not a memset: callers may capture this stream)
    QW_HIP(qw::launch_fill(lam.rbuf[0], int64_t(2 * planes), stream));
    QW_HIP(qw::launch_fill(gb.dw, int64_t(up(sizeof(double) * size_t(ctx->jtotal))), stream));
    int64_t src = 0;
    for (int32_t i = 0; i < ctx->ninst; ++i) {
      const HostInst& hi = ctx->inst[i];
      QW_HIP(hipMemcpyAsync(gb.dw + hi.jbase, w + src, sizeof(double) * hi.n, hipMemcpyHostToDevice, stream));
      src += hi.n;
    }
    rc = grad_sweep(st, &lam, true, gb, nsteps, dvals, nullptr, db_re, db_im, loss, stream);
    (void)hipStreamSynchronize(stream);
    return rc;
  });
}

}  // extern "C"
