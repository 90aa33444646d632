// Internal declarations shared by the host API (qw_api.cpp), the launchers
// (qw_launch.cpp) and the kernels (qw_kernels.hip) of libqw.  Not part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace qw {

constexpr int kWave = 64;       // CDNA wavefront width
constexpr int kMaxS = 64;       // largest QRAM row length handled (one wave per group)
constexpr int kMaxGrid = 65536;  // largest step-kernel grid
constexpr int kMaxBlock = 256;  // largest step-kernel workgroup
constexpr int kMaxWaves = kMaxGrid * (kMaxBlock / kWave);  // per-wavefront counters
// Lanes per row of the step kernels: min(s, 8), or 16 for s >= 16 when the
// context then has at most kWideWaves wavefronts (Matrix::wide): more,
// shorter lanes for a launch that would not fill the chip.
constexpr int kWideWaves = 2048;
constexpr double kTau = 1e-13;  // pruning threshold applied after every step
// Size of the device array `scratch` of the code object (one per device,
// from the code object's load to qw_shutdown): the buffers of
// qw_grad_noalloc.
constexpr size_t kScratchBytes = size_t(32) << 20;
// Keys per workgroup of the export's radix-sort passes (256 threads, 8 keys each).
constexpr int kSortTile = 256 * 8;

// Per-instance facts, resident on the device.  The slots of instance i are
// [item_base, item_base + N*s); the base is a multiple of 64 so that a
// wavefront of a pass over slots never straddles two instances.  The ELL
// arrays col/val hold slot (j, l) at item_base + j*s + l (row-major, for the
// binary searches); the state planes and the slot records hold it at its
// home item_base + l*N + j.
struct Inst {
  int64_t item_base;  // first slot
  int64_t jbase;      // offset of this instance in N-vectors
  int64_t wave_base;  // first wavefront of this instance in the step kernels
  int32_t N;          // padded dimension (power of two)
  int32_t s;          // slots per row (power of two, <= 64)
  int32_t hbits;      // log2 s
  int32_t nlog;       // log2 N
  int32_t lpr_log;    // log2 of the lanes that share a row in the step kernels: min(s, 8)
  int32_t sl;         // slots per lane there: s / min(s, 8)
  double inv_sqrt_s;  // 1/sqrt(s)
};

// Amplitudes with a static home, four planes indexed by home h of slot
// q = (j, l):
//   R0[h], R1[h]: key K(q, b2) = (0, j, 0, 0, col[q], b2)    (group members)
//   Q0[h], Q1[h]: key S K(q, b2) = (0, col[q], b2, 0, j, 0)  when it is not
//                 itself a group member (always for b2 = 1; for b2 = 0 only
//                 when j is absent from row col[q]); Q0 stays 0 otherwise.
// Complex double; an exact 0 means "no branch".  A state owns R0, Q0 and Q1
// planes in each of two parity buffers; the view of the state in buffer p
// takes R1 from buffer 1-p's Q1 plane, which holds r1s * R1 (r1s = +-1).
struct Slots {
  double2* R0;
  double2* R1;
  double2* Q0;
  double2* Q1;
  double r1s;  // the R1 plane holds r1s * R1
};

// Branches outside the span of those keys (imports, raw starts): the walk
// maps each to -S(key), so the list keeps its size and order.
struct List {
  uint64_t* key;
  double2* amp;
  uint32_t cnt;
  uint32_t cap;
};

// What the step reads of a slot, in one 16-byte load at the slot's home.
struct SlotRec {
  int32_t col;   // column index col[q]
  int32_t part;  // home of K(q', 0) relative to item_base (q' = (col[q], rev[q])), or -1
  double val;    // a_{j,l} after scaling
};

// Fixed-point data (angles = 1): the value of a slot is replaced by the
// signed angle y (in units of pi, |y| <= 1/2) of its conditional rotation,
// f = sin(pi |y|) (times +-i when y < 0), g = cos(pi y); a zero value has
// y = 0 (f = 0, g = 1).
struct Matrix {
  const int32_t* col;        // ELL column indices (row-major), sorted inside each row
  const double* val;         // ELL values (row-major)
  const SlotRec* rec;        // slot records (by home)
  // What the step kernels read of a slot (12 bytes, by home, two planes so
  // that a wavefront's eight-row runs stay sector-aligned): slink bits 0-30
  // hold part + 1 (0: no partner) and bit 31 is set when row j > column
  // col[q], the one fact of the column that the rule for negative values
  // needs; sval is the value.
  const uint32_t* slink;
  const double* sval;
  // The rotation of every slot, computed once at load exactly as the step
  // kernels compute it (qwk_rot_table), by home.  Real matrices (realsym):
  // two doubles, f' (the +-i rule's sign taken into f for a negative value)
  // and g, read by the one-double-per-cell kernels of one s with at most two
  // slots per lane in place of sval and two square roots.  Complex values:
  // four doubles, f (real, imaginary), g and 0, read by the complex kernels
  // of one s with at most two slots per lane in place of sval, vim and the
  // principal square root.  NULL otherwise.
  const double* sfg;
  const double* vim;         // imaginary parts of the values by home (NULL: a real matrix)
  const Inst* inst;
  const int32_t* wave_inst;  // instance of every step-kernel wavefront
  int64_t items;             // total slots including alignment padding
  int64_t waves;             // wavefronts of one step-kernel pass
  int64_t rows;              // sum of N over the instances (length of N-vectors)
  int32_t ninst;
  int32_t nbits;             // register width n of the key layout
  int32_t smax;              // largest s over the instances
  int32_t slmax;             // largest slots-per-lane over the instances
  int32_t suni;              // s of every instance when they all share it, else 0
  int16_t full;  // 1 when every instance has at least one wavefront of rows
  // Row blocks of the one-pass step and adjoint kernels numbered by XCD
  // (xcd_row_block, the _x kernels): -1 in the context's matrix when it was
  // loaded with QW_XCD_ROWS; launch_step and launch_adjoint replace it by the
  // launch's workgroups per XCD (grid / 8; 0, the plain numbering, for a grid
  // that is not a multiple of 8), pick the _x kernels when it is positive and
  // pass it to them in the upper bits of wpb.
  int16_t xcd;
  int32_t angles;            // 1: fixed-point data; val holds each slot's rotation angle (below)
  int32_t wide;              // 1: instances with s >= 16 use 16 lanes per row (kWideWaves)
  Inst inst0;                // copy of inst[0] (a single instance needs no table read)
};

enum Mode : int32_t { kStep = 0, kSwap = 1 };
// What a slot's value is, for the step kernels' rotation.
enum Enc : int32_t { kEncReal = 0, kEncComplex = 1, kEncAngle = 2 };

struct StepArgs {
  Matrix m;
  Slots in, out;
  List L;
  unsigned long long* acc;  // running counts of kept outputs (a Q1 output twice), kMaxWaves entries,
                            // or NULL: no counts (a walk whose counts nobody reads)
  int32_t mode;             // kStep: W; kSwap: S only
  int32_t wpb;              // wavefronts per workgroup (set by the launcher); for the _x kernels
                            // bits 8 and up hold the workgroups per XCD (xcd_row_block)
  double tau;
  // optional fused projection (linear solver): y[j] += coef[0] <psi~_j|state>,
  // coef pointing at this launch's coefficient (its entry of the host's table,
  // or inside a graph an entry of a window that a node ahead of the steps
  // refreshes on every replay: qwk_coef_window)
  double2* yacc;
  const double* coef;
  // 1: every slot of value 0 has R0 = 0 (and Q0 = 0) in this state and its
  // partner is a slot of value 0 too, so the grid-stride and g kernels skip
  // those cells of such slots (they stay 0 under the step and the swap)
  int32_t zskip;
  // 1: one double per cell (real amplitudes, or imaginary ones in the R0
  // cells of slots of negative value); the plane pointers of in/out point at
  // double arrays (the qwk_step_r / qwk_step_t kernels)
  int32_t real;
  // 1: some slot has no partner (Matrix::q0): the launcher takes the real
  // kernels' _q forms, which read Q0 of such slots with the other loads
  // (step_wave_real's EQ0); the kernels do not read it
  int32_t q0;
};

struct AdjArgs {
  Matrix m;
  Slots in, out;    // recomputed state (kept S-conjugated)
  Slots lin, lout;  // adjoint state (kept S-conjugated)
  List L, LL;
  unsigned long long* acc;
  unsigned long long* lacc;
  double tau;
  double* dv;       // gradient per slot (by home), accumulated
  int32_t wpb;      // wavefronts per workgroup (set by the launcher; bits 8 and up as StepArgs::wpb)
  // 1: both states on one double per cell (the plane pointers point at
  // double arrays; the qwk_adjoint_r kernels: one pass, empty lists)
  int32_t real;
  int32_t q0;  // as StepArgs::q0
  // dL/d(Im v) per slot (by home), accumulated: complex values only (the
  // complex-plane kernels with Matrix::vim), NULL otherwise; dv then holds
  // dL/d(Re v).
  double* dvi;
};

// The host side is compiled by the host compiler and the kernels by the GPU
// compiler; the argument structures must have one layout on both.
static_assert(sizeof(Inst) == 56 && offsetof(Inst, inv_sqrt_s) == 48, "Inst layout");
static_assert(sizeof(Slots) == 40 && offsetof(Slots, r1s) == 32, "Slots layout");
static_assert(sizeof(List) == 24 && offsetof(List, cap) == 20, "List layout");
static_assert(sizeof(SlotRec) == 16 && offsetof(SlotRec, val) == 8, "SlotRec layout");
static_assert(sizeof(Matrix) == 184 && offsetof(Matrix, inst0) == 128, "Matrix layout");
static_assert(sizeof(StepArgs) == 344 && offsetof(StepArgs, zskip) == 328 && offsetof(StepArgs, q0) == 336,
              "StepArgs layout");
static_assert(sizeof(AdjArgs) == 448 && offsetof(AdjArgs, wpb) == 424 && offsetof(AdjArgs, q0) == 432 &&
                  offsetof(AdjArgs, dvi) == 440,
              "AdjArgs layout");

// The current device's `scratch` array: its device address and size, looked
// up on that device's module when the module is loaded (qw_launch.cpp).
hipError_t device_scratch(void** ptr, size_t* bytes);

// Launchers (qw_launch.cpp).  All enqueue on `stream` and allocate nothing.
hipError_t launch_step(const StepArgs& a, int grid, int block, hipStream_t stream);
hipError_t launch_adjoint(const AdjArgs& a, int grid, int block, hipStream_t stream);
// Slot records of both kinds (the QBS of every reflected output, once per matrix).
hipError_t launch_qbs_table(const Matrix& m, SlotRec* rec, uint32_t* slink, double* sval, hipStream_t stream);
// Fill Matrix::sfg (2 doubles per slot) from slink and sval (after launch_qbs_table).
hipError_t launch_rot_table(const Matrix& m, double* sfg, hipStream_t stream);
hipError_t launch_init(const Matrix& m, const double2* b, Slots out, double tau, hipStream_t stream);
hipError_t launch_fill(void* p, int64_t bytes, hipStream_t stream);
// out[0 .. kSumBlocks) = partial sums of a[0 .. n) (the per-wavefront counters).
constexpr int kSumBlocks = 256;
hipError_t launch_sum_counts(const unsigned long long* a, int64_t n, unsigned long long* out, hipStream_t stream);
// window[i] = table[*base + i] for i < count, then *base += count; with
// set >= 0 only *base = set.
hipError_t launch_coef_window(const double* table, int64_t* base, double* window, int32_t count, int64_t set,
                              hipStream_t stream);
// n complex cells to the one double each holds, and back: the imaginary part
// where val (by cell, or NULL) is negative, the real part elsewhere.
hipError_t launch_to_real(const double2* src, double* dst, const double* val, int64_t n, hipStream_t stream);
hipError_t launch_to_complex(const double* src, double2* dst, const double* val, int64_t n, hipStream_t stream);
// Reductions over a state: kind 0 = count, 1 = norm^2, 4 = count of the Q1
// plane (per-block partials in `partial`, length >= grid); kind 2 = j
// marginal into out (N-vector, must be zero); kind 3 = projection
// <psi~_j|state> into out (interleaved complex).  `grid` applies to kinds 0,
// 1 and 4.
hipError_t launch_measure(const Matrix& m, Slots st, List L, int32_t kind, double* partial, double* out, int grid,
                          hipStream_t stream);
hipError_t launch_export(const Matrix& m, Slots st, List L, uint64_t* keys, double2* amps, uint32_t* count,
                         uint32_t cap, hipStream_t stream);
// The export's key order.  launch_key_bits: bits[0] |= OR of keys[0 .. count),
// bits[1] |= OR of their complements (bits[] zeroed by the caller).
// launch_radix_pass: one stable counting-sort pass on the 8-bit digit at
// `shift` moving (kin, vin) to (kout, vout); hist holds 256 counters per tile
// of kSortTile keys, digit_base 256.
hipError_t launch_key_bits(const uint64_t* keys, int64_t count, unsigned long long* bits, hipStream_t stream);
hipError_t launch_radix_pass(const uint64_t* kin, const double2* vin, int64_t count, int shift, uint32_t* hist,
                             uint32_t* digit_base, uint64_t* kout, double2* vout, hipStream_t stream);
// re[i], im[i] = a[i] for i < n.
hipError_t launch_split_amps(const double2* a, int64_t n, double* re, double* im, hipStream_t stream);
// Place unique branches at their homes; keys with no static home are appended
// to the list (count in *lcnt, which must start at 0).
hipError_t launch_import(const Matrix& m, const uint64_t* keys, const double2* amps, int64_t n, Slots out, List L,
                         uint32_t* lcnt, hipStream_t stream);
hipError_t launch_weight(const Matrix& m, Slots in, List L, Slots out, List LL, const double* w, double* partial,
                         int grid, hipStream_t stream);
// dvi: dL/d(Im v) by home for complex values (Matrix::vim), NULL otherwise.
hipError_t launch_grad_init(const Matrix& m, Slots lam, const double2* b, double* dv, double2* db, double* dvi,
                            hipStream_t stream);
// The same three on one double per cell (the plane pointers point at double
// arrays): the swap S (counted into acc unless NULL), the weighting, and the
// gradient through the initial T~ for a real b.
hipError_t launch_swap_real(const Matrix& m, Slots in, Slots out, unsigned long long* acc, hipStream_t stream);
hipError_t launch_weight_real(const Matrix& m, Slots in, Slots out, const double* w, double* partial, int grid,
                              hipStream_t stream);
hipError_t launch_grad_init_real(const Matrix& m, Slots lam, const double2* b, double* dv, double2* db,
                                 hipStream_t stream);
// gv[p] = dv[home[p]] (p < nnz) and br/bi[p] = db[row[p]] (p < n); with
// dvi (complex values) also gvi[p] = dvi[home[p]].
hipError_t launch_gather_grad(const double* dv, const int32_t* home, int64_t nnz, const double2* db,
                              const int32_t* row, int64_t n, double* gv, double* br, double* bi,
                              const double* dvi, double* gvi, hipStream_t stream);

}  // namespace qw
