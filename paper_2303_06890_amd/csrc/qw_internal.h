// Internal declarations shared by the host API (qw_api.hip) and the kernels
// (qw_kernels.hip) of libqw.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace qw {

constexpr int kWave = 64;      // CDNA wavefront width
constexpr int kMaxS = 64;      // largest QRAM row length handled (one wave per group)
constexpr double kTau = 1e-13;  // pruning threshold applied after every step

// Per-instance facts, resident on the device.  The reflection slots of
// instance i are the ELL entries [item_base, item_base + N*s); the base is a
// multiple of 64 so that a wavefront never straddles two instances.
struct Inst {
  int64_t item_base;  // first ELL slot (= first phase-A work item)
  int64_t jbase;      // offset of this instance in N-vectors
  int32_t N;          // padded dimension (power of two)
  int32_t s;          // slots per row (power of two, <= 64)
  int32_t hbits;      // log2 s
  int32_t pad_;
  double inv_sqrt_s;  // 1/sqrt(s)
};

// One branch list (the sparse part of a state) plus its reflection-slot
// array.  R holds, for every ELL slot q = (inst, j, l), the amplitudes of the
// two keys (0, j, 0, 0, col[q], b2), b2 = 0 at R[2q] and b2 = 1 at R[2q+1]
// (interleaved complex double).  Every other branch lives in the list.
struct Buf {
  double2* R;
  uint64_t* key;
  double2* amp;
  uint32_t* cnt;  // number of list entries (may exceed cap after an overflow)
  uint32_t cap;   // list capacity
};

// Device-side bookkeeping of a state (one cache line each to avoid sharing).
struct Ctl {
  uint32_t cnt[2];         // list counts of the two buffers
  uint32_t pad0[30];
  uint32_t done;           // workgroups finished in the current launch
  uint32_t pad1[31];
  uint32_t overflow;       // set when a list append exceeded the capacity
  uint32_t pad2[31];
  unsigned long long written;       // branches kept by the current launch
  unsigned long long last_written;  // ... by the last completed launch
  unsigned long long steps;         // completed step launches
  unsigned long long total_written; // branches kept, summed over all launches
  uint32_t stepno;                  // solver step counter (indexes the coefficient table)
  uint32_t pad3[23];
};

struct Matrix {
  const int32_t* col;  // ELL column indices, sorted inside each row
  const double* val;   // ELL values
  const Inst* inst;
  int32_t ninst;
  int32_t nbits;       // register width n of the key layout
  int64_t items;       // total ELL slots including alignment padding
};

enum Mode : int32_t { kStep = 0, kSwap = 1 };

struct StepArgs {
  Matrix m;
  Buf in, out;
  Ctl* ctl;
  uint32_t cap;
  int32_t mode;
  double tau;
  // optional fused projection accumulation (linear solver): y[j] += coefm[stepno] * <psi~_j|state>
  double2* yacc;
  const double* coefm;
};

struct AdjArgs {
  Matrix m;
  Buf in, out;    // the recomputed state
  Buf lin, lout;  // the adjoint state
  Ctl* ctl;
  Ctl* lctl;
  uint32_t cap;
  double tau;
  double* dv;     // gradient per ELL slot, accumulated
};

// The host side is compiled by the host compiler and the kernels by the GPU
// compiler; the argument structures must have one layout on both.
static_assert(sizeof(Inst) == 40 && offsetof(Inst, inv_sqrt_s) == 32, "Inst layout");
static_assert(sizeof(Buf) == 40 && offsetof(Buf, cap) == 32, "Buf layout");
static_assert(sizeof(Matrix) == 40 && offsetof(Matrix, items) == 32, "Matrix layout");
static_assert(sizeof(StepArgs) == 160 && offsetof(StepArgs, coefm) == 152, "StepArgs layout");
static_assert(sizeof(AdjArgs) == 240 && offsetof(AdjArgs, dv) == 232, "AdjArgs layout");

// Launchers (qw_launch.cpp).  All enqueue on `stream` and allocate nothing.
hipError_t launch_step(const StepArgs& a, int grid, int block, hipStream_t stream);
hipError_t launch_adjoint(const AdjArgs& a, int grid, int block, hipStream_t stream);
hipError_t launch_init(const Matrix& m, const double2* b, Buf out, Ctl* ctl, uint32_t cap, int32_t raw,
                       double tau, hipStream_t stream);
hipError_t launch_fill(void* p, int64_t bytes, hipStream_t stream);
// Reductions over a state: kind 0 = count, 1 = norm^2 (per-block partials
// in `partial`, length >= grid), 2 = j marginal (atomics into out[N-vector]),
// 3 = projection <psi~_j|state> into out (interleaved complex).
hipError_t launch_measure(const Matrix& m, Buf b, int32_t kind, double* partial, double* out, int grid,
                          hipStream_t stream);
hipError_t launch_export(const Matrix& m, Buf b, uint64_t* keys, double2* amps, uint32_t* count,
                         uint32_t cap, hipStream_t stream);
hipError_t launch_import(const Matrix& m, const uint64_t* keys, const double2* amps, int64_t n, Buf out,
                         Ctl* ctl, uint32_t cap, hipStream_t stream);
hipError_t launch_weight(const Matrix& m, Buf in, Buf out, Ctl* octl, const double* w, uint32_t cap,
                         double* partial, int grid, hipStream_t stream);
hipError_t launch_grad_init(const Matrix& m, Buf lam, const double2* b, double* dv, double2* db,
                            hipStream_t stream);

}  // namespace qw
