// Host launchers of libqw's kernels.
//
// The kernels are compiled into a separate gfx950 code object that is
// embedded in libqw.so (qw_code_object, generated at build time) and loaded
// into the HIP runtime explicitly, once per device, on first use
// (hipModuleLoadData); qw_shutdown() unloads it.  The library therefore holds
// no compiler-generated static registration of device code: what it puts into
// the runtime is created and released by explicit calls, independent of the
// order in which a process tears down its runtime(s) at exit.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/qw.h"
#include "qw_internal.h"

extern "C" const unsigned char qw_code_object[];
extern "C" const size_t qw_code_object_size;

namespace qw {
namespace {

// Step kernels: qwk_step_s{1,2,4,8} take any s per instance with up to that
// many slots held per lane (s <= 8, 16, 32, 64), any launch shape and either
// mode; qwk_step_g{1,2,4,8} need every instance to have at least one
// wavefront's rows, a grid that covers the work in one pass, and the walk
// step; qwk_step_f{S} need that and s = S for every instance;
// qwk_step_c{1,2,4,8} are the general kernels for complex Hermitian matrices
// and qwk_step_x{1,2,4,8} those for fixed-point data, qwk_step_h{1,2,4,8} and
// qwk_step_y{1,2,4,8} their one-pass forms (the conditions of the g
// kernels); qwk_step_k{S} is the complex form of the f kernels.  Each has an _acc twin
// (the solver's fused projection).  Adjoint kernels (real FP64 matrices) come
// in the four widths.  qwk_step_r{S} and qwk_step_t{S} are the f kernels on
// one double per cell (8-byte planes), FP64 and fixed-point values, and
// qwk_step_rg{N} and qwk_step_tg{N} the g kernels on them; each has an _acc
// twin too.
enum Fn {
  F_STEP_S1,
  F_STEP_S2,
  F_STEP_S4,
  F_STEP_S8,
  F_STEP_G1,
  F_STEP_G2,
  F_STEP_G4,
  F_STEP_G8,
  F_STEP_F1,
  F_STEP_F2,
  F_STEP_F4,
  F_STEP_F8,
  F_STEP_F16,
  F_STEP_F32,
  F_STEP_F64,
  F_STEP_C1,
  F_STEP_C2,
  F_STEP_C4,
  F_STEP_C8,
  F_STEP_X1,
  F_STEP_X2,
  F_STEP_X4,
  F_STEP_X8,
  F_STEP_H1,
  F_STEP_H2,
  F_STEP_H4,
  F_STEP_H8,
  F_STEP_Y1,
  F_STEP_Y2,
  F_STEP_Y4,
  F_STEP_Y8,
  F_STEP_K1,  // complex values, s = 1 ... 64 for every instance: qwk_step_k{1..64}
  F_STEP_FW16 = F_STEP_K1 + 7,  // 16 lanes per row (Matrix::wide): qwk_step_f{16,32,64}w,
  F_STEP_KW16 = F_STEP_FW16 + 3,  // then qwk_step_k{16,32,64}w
  F_STEP_COUNT_ = F_STEP_KW16 + 3,  // _acc twins follow at + F_STEP_COUNT_
  F_ADJOINT_S1 = 2 * F_STEP_COUNT_,
  F_ADJOINT_S2,
  F_ADJOINT_S4,
  F_ADJOINT_S8,
  F_QBS_TABLE,
  F_INIT,
  F_FILL,
  F_MEASURE,
  F_MEASURE_ROWS,
  F_EXPORT,
  F_IMPORT,
  F_WEIGHT,
  F_GRAD_INIT,
  F_STEP_R1,  // one double per cell: qwk_step_r{1..64}, qwk_step_t{1..64}, then mixed s:
  F_STEP_T1 = F_STEP_R1 + 7,    // qwk_step_rg{1,2,4,8}, qwk_step_tg{1,2,4,8}; their _acc
  F_STEP_RG1 = F_STEP_T1 + 7,   // twins follow at + F_REAL_COUNT_, the _q forms (early Q0
  F_STEP_TG1 = F_STEP_RG1 + 4,  // loads) at + 2 F_REAL_COUNT_ and their _acc twins at
  F_STEP_RW16 = F_STEP_TG1 + 4,  // + 3 F_REAL_COUNT_.  16 lanes per row: qwk_step_r{16,32,64}w,
  F_STEP_TW16 = F_STEP_RW16 + 3,  // qwk_step_t{16,32,64}w
  F_REAL_COUNT_ = F_STEP_TW16 + 3 - F_STEP_R1,
  F_TO_REAL = F_STEP_R1 + 8 * F_REAL_COUNT_,  // + 4 F_REAL_COUNT_: the _x forms (row blocks by XCD)
  F_TO_COMPLEX,
  F_COEF_WINDOW,
  F_SUM_COUNTS,
  F_ADJ_R1,                   // one-pass adjoint on one double per cell: qwk_adjoint_r{1..64},
  F_ADJ_RG1 = F_ADJ_R1 + 7,   // qwk_adjoint_rg{1,2,4,8} (mixed s),
  F_ADJ_RW16 = F_ADJ_RG1 + 4,  // qwk_adjoint_r{16,32,64}w (16 lanes per row); the _q forms
  F_ADJ_COUNT_ = F_ADJ_RW16 + 3 - F_ADJ_R1,  // follow at + F_ADJ_COUNT_, the _x forms (row blocks by
                                             // XCD) at + 2 F_ADJ_COUNT_ and their _q forms at + 3
  F_SWAP_REAL = F_ADJ_R1 + 4 * F_ADJ_COUNT_,
  F_WEIGHT_REAL,
  F_GRAD_INIT_REAL,
  F_GATHER_GRAD,
  F_ROT_TABLE,
  F_KEY_BITS,
  F_RADIX_HIST,
  F_RADIX_OFFSETS,
  F_RADIX_SCATTER,
  F_SPLIT_AMPS,
  F_COUNT
};

const char* const kNames[] = {
    "qwk_step_s1",      "qwk_step_s2",      "qwk_step_s4",      "qwk_step_s8",      "qwk_step_g1",
    "qwk_step_g2",      "qwk_step_g4",      "qwk_step_g8",      "qwk_step_f1",      "qwk_step_f2",
    "qwk_step_f4",      "qwk_step_f8",      "qwk_step_f16",     "qwk_step_f32",     "qwk_step_f64",
    "qwk_step_c1",      "qwk_step_c2",      "qwk_step_c4",      "qwk_step_c8",      "qwk_step_x1",
    "qwk_step_x2",      "qwk_step_x4",      "qwk_step_x8",      "qwk_step_h1",      "qwk_step_h2",
    "qwk_step_h4",      "qwk_step_h8",      "qwk_step_y1",      "qwk_step_y2",      "qwk_step_y4",
    "qwk_step_y8",      "qwk_step_k1",      "qwk_step_k2",      "qwk_step_k4",      "qwk_step_k8",
    "qwk_step_k16",     "qwk_step_k32",     "qwk_step_k64",     "qwk_step_f16w",    "qwk_step_f32w",
    "qwk_step_f64w",    "qwk_step_k16w",    "qwk_step_k32w",    "qwk_step_k64w",
    "qwk_step_s1_acc",  "qwk_step_s2_acc",  "qwk_step_s4_acc",  "qwk_step_s8_acc",  "qwk_step_g1_acc",
    "qwk_step_g2_acc",  "qwk_step_g4_acc",  "qwk_step_g8_acc",  "qwk_step_f1_acc",  "qwk_step_f2_acc",
    "qwk_step_f4_acc",  "qwk_step_f8_acc",  "qwk_step_f16_acc", "qwk_step_f32_acc", "qwk_step_f64_acc",
    "qwk_step_c1_acc",  "qwk_step_c2_acc",  "qwk_step_c4_acc",  "qwk_step_c8_acc",  "qwk_step_x1_acc",
    "qwk_step_x2_acc",  "qwk_step_x4_acc",  "qwk_step_x8_acc",  "qwk_step_h1_acc",  "qwk_step_h2_acc",
    "qwk_step_h4_acc",  "qwk_step_h8_acc",  "qwk_step_y1_acc",  "qwk_step_y2_acc",  "qwk_step_y4_acc",
    "qwk_step_y8_acc",  "qwk_step_k1_acc",  "qwk_step_k2_acc",  "qwk_step_k4_acc",  "qwk_step_k8_acc",
    "qwk_step_k16_acc", "qwk_step_k32_acc", "qwk_step_k64_acc", "qwk_step_f16w_acc", "qwk_step_f32w_acc",
    "qwk_step_f64w_acc", "qwk_step_k16w_acc", "qwk_step_k32w_acc", "qwk_step_k64w_acc",
    "qwk_adjoint_s1",   "qwk_adjoint_s2",   "qwk_adjoint_s4",   "qwk_adjoint_s8",   "qwk_qbs_table",
    "qwk_init",         "qwk_fill",         "qwk_measure",      "qwk_measure_rows", "qwk_export",
    "qwk_import",       "qwk_weight",       "qwk_grad_init",    "qwk_step_r1",      "qwk_step_r2",
    "qwk_step_r4",      "qwk_step_r8",      "qwk_step_r16",     "qwk_step_r32",     "qwk_step_r64",
    "qwk_step_t1",      "qwk_step_t2",      "qwk_step_t4",      "qwk_step_t8",      "qwk_step_t16",
    "qwk_step_t32",     "qwk_step_t64",     "qwk_step_rg1",     "qwk_step_rg2",     "qwk_step_rg4",
    "qwk_step_rg8",     "qwk_step_tg1",     "qwk_step_tg2",     "qwk_step_tg4",     "qwk_step_tg8",
    "qwk_step_r16w",    "qwk_step_r32w",    "qwk_step_r64w",    "qwk_step_t16w",    "qwk_step_t32w",
    "qwk_step_t64w",
    "qwk_step_r1_acc",  "qwk_step_r2_acc",  "qwk_step_r4_acc",  "qwk_step_r8_acc",  "qwk_step_r16_acc",
    "qwk_step_r32_acc", "qwk_step_r64_acc", "qwk_step_t1_acc",  "qwk_step_t2_acc",  "qwk_step_t4_acc",
    "qwk_step_t8_acc",  "qwk_step_t16_acc", "qwk_step_t32_acc", "qwk_step_t64_acc", "qwk_step_rg1_acc",
    "qwk_step_rg2_acc", "qwk_step_rg4_acc", "qwk_step_rg8_acc", "qwk_step_tg1_acc", "qwk_step_tg2_acc",
    "qwk_step_tg4_acc", "qwk_step_tg8_acc", "qwk_step_r16w_acc", "qwk_step_r32w_acc", "qwk_step_r64w_acc",
    "qwk_step_t16w_acc", "qwk_step_t32w_acc", "qwk_step_t64w_acc",
    "qwk_step_r1_q", "qwk_step_r2_q", "qwk_step_r4_q", "qwk_step_r8_q", "qwk_step_r16_q", "qwk_step_r32_q",
    "qwk_step_r64_q", "qwk_step_t1_q", "qwk_step_t2_q", "qwk_step_t4_q", "qwk_step_t8_q", "qwk_step_t16_q",
    "qwk_step_t32_q", "qwk_step_t64_q", "qwk_step_rg1_q", "qwk_step_rg2_q", "qwk_step_rg4_q",
    "qwk_step_rg8_q", "qwk_step_tg1_q", "qwk_step_tg2_q", "qwk_step_tg4_q", "qwk_step_tg8_q",
    "qwk_step_r16w_q", "qwk_step_r32w_q", "qwk_step_r64w_q", "qwk_step_t16w_q", "qwk_step_t32w_q",
    "qwk_step_t64w_q",
    "qwk_step_r1_q_acc", "qwk_step_r2_q_acc", "qwk_step_r4_q_acc", "qwk_step_r8_q_acc", "qwk_step_r16_q_acc",
    "qwk_step_r32_q_acc", "qwk_step_r64_q_acc", "qwk_step_t1_q_acc", "qwk_step_t2_q_acc", "qwk_step_t4_q_acc",
    "qwk_step_t8_q_acc", "qwk_step_t16_q_acc", "qwk_step_t32_q_acc", "qwk_step_t64_q_acc",
    "qwk_step_rg1_q_acc", "qwk_step_rg2_q_acc", "qwk_step_rg4_q_acc", "qwk_step_rg8_q_acc",
    "qwk_step_tg1_q_acc", "qwk_step_tg2_q_acc", "qwk_step_tg4_q_acc", "qwk_step_tg8_q_acc",
    "qwk_step_r16w_q_acc", "qwk_step_r32w_q_acc", "qwk_step_r64w_q_acc", "qwk_step_t16w_q_acc",
    "qwk_step_t32w_q_acc", "qwk_step_t64w_q_acc",
    "qwk_step_r1_x", "qwk_step_r2_x", "qwk_step_r4_x", "qwk_step_r8_x",
    "qwk_step_r16_x", "qwk_step_r32_x", "qwk_step_r64_x", "qwk_step_t1_x",
    "qwk_step_t2_x", "qwk_step_t4_x", "qwk_step_t8_x", "qwk_step_t16_x",
    "qwk_step_t32_x", "qwk_step_t64_x", "qwk_step_rg1_x", "qwk_step_rg2_x",
    "qwk_step_rg4_x", "qwk_step_rg8_x", "qwk_step_tg1_x", "qwk_step_tg2_x",
    "qwk_step_tg4_x", "qwk_step_tg8_x", "qwk_step_r16w_x", "qwk_step_r32w_x",
    "qwk_step_r64w_x", "qwk_step_t16w_x", "qwk_step_t32w_x", "qwk_step_t64w_x",
    "qwk_step_r1_x_acc", "qwk_step_r2_x_acc", "qwk_step_r4_x_acc", "qwk_step_r8_x_acc",
    "qwk_step_r16_x_acc", "qwk_step_r32_x_acc", "qwk_step_r64_x_acc", "qwk_step_t1_x_acc",
    "qwk_step_t2_x_acc", "qwk_step_t4_x_acc", "qwk_step_t8_x_acc", "qwk_step_t16_x_acc",
    "qwk_step_t32_x_acc", "qwk_step_t64_x_acc", "qwk_step_rg1_x_acc", "qwk_step_rg2_x_acc",
    "qwk_step_rg4_x_acc", "qwk_step_rg8_x_acc", "qwk_step_tg1_x_acc", "qwk_step_tg2_x_acc",
    "qwk_step_tg4_x_acc", "qwk_step_tg8_x_acc", "qwk_step_r16w_x_acc", "qwk_step_r32w_x_acc",
    "qwk_step_r64w_x_acc", "qwk_step_t16w_x_acc", "qwk_step_t32w_x_acc", "qwk_step_t64w_x_acc",
    "qwk_step_r1_x_q", "qwk_step_r2_x_q", "qwk_step_r4_x_q", "qwk_step_r8_x_q",
    "qwk_step_r16_x_q", "qwk_step_r32_x_q", "qwk_step_r64_x_q", "qwk_step_t1_x_q",
    "qwk_step_t2_x_q", "qwk_step_t4_x_q", "qwk_step_t8_x_q", "qwk_step_t16_x_q",
    "qwk_step_t32_x_q", "qwk_step_t64_x_q", "qwk_step_rg1_x_q", "qwk_step_rg2_x_q",
    "qwk_step_rg4_x_q", "qwk_step_rg8_x_q", "qwk_step_tg1_x_q", "qwk_step_tg2_x_q",
    "qwk_step_tg4_x_q", "qwk_step_tg8_x_q", "qwk_step_r16w_x_q", "qwk_step_r32w_x_q",
    "qwk_step_r64w_x_q", "qwk_step_t16w_x_q", "qwk_step_t32w_x_q", "qwk_step_t64w_x_q",
    "qwk_step_r1_x_q_acc", "qwk_step_r2_x_q_acc", "qwk_step_r4_x_q_acc", "qwk_step_r8_x_q_acc",
    "qwk_step_r16_x_q_acc", "qwk_step_r32_x_q_acc", "qwk_step_r64_x_q_acc", "qwk_step_t1_x_q_acc",
    "qwk_step_t2_x_q_acc", "qwk_step_t4_x_q_acc", "qwk_step_t8_x_q_acc", "qwk_step_t16_x_q_acc",
    "qwk_step_t32_x_q_acc", "qwk_step_t64_x_q_acc", "qwk_step_rg1_x_q_acc", "qwk_step_rg2_x_q_acc",
    "qwk_step_rg4_x_q_acc", "qwk_step_rg8_x_q_acc", "qwk_step_tg1_x_q_acc", "qwk_step_tg2_x_q_acc",
    "qwk_step_tg4_x_q_acc", "qwk_step_tg8_x_q_acc", "qwk_step_r16w_x_q_acc", "qwk_step_r32w_x_q_acc",
    "qwk_step_r64w_x_q_acc", "qwk_step_t16w_x_q_acc", "qwk_step_t32w_x_q_acc", "qwk_step_t64w_x_q_acc",
    "qwk_to_real",      "qwk_to_complex",
    "qwk_coef_window",  "qwk_sum_counts",
    "qwk_adjoint_r1",   "qwk_adjoint_r2",   "qwk_adjoint_r4",   "qwk_adjoint_r8",   "qwk_adjoint_r16",
    "qwk_adjoint_r32",  "qwk_adjoint_r64",  "qwk_adjoint_rg1",  "qwk_adjoint_rg2",  "qwk_adjoint_rg4",
    "qwk_adjoint_rg8",  "qwk_adjoint_r16w", "qwk_adjoint_r32w", "qwk_adjoint_r64w",
    "qwk_adjoint_r1_q", "qwk_adjoint_r2_q", "qwk_adjoint_r4_q", "qwk_adjoint_r8_q", "qwk_adjoint_r16_q",
    "qwk_adjoint_r32_q", "qwk_adjoint_r64_q", "qwk_adjoint_rg1_q", "qwk_adjoint_rg2_q", "qwk_adjoint_rg4_q",
    "qwk_adjoint_rg8_q", "qwk_adjoint_r16w_q", "qwk_adjoint_r32w_q", "qwk_adjoint_r64w_q",
    "qwk_adjoint_r1_x", "qwk_adjoint_r2_x", "qwk_adjoint_r4_x", "qwk_adjoint_r8_x",
    "qwk_adjoint_r16_x", "qwk_adjoint_r32_x", "qwk_adjoint_r64_x", "qwk_adjoint_rg1_x",
    "qwk_adjoint_rg2_x", "qwk_adjoint_rg4_x", "qwk_adjoint_rg8_x", "qwk_adjoint_r16w_x",
    "qwk_adjoint_r32w_x", "qwk_adjoint_r64w_x", "qwk_adjoint_r1_x_q", "qwk_adjoint_r2_x_q",
    "qwk_adjoint_r4_x_q", "qwk_adjoint_r8_x_q", "qwk_adjoint_r16_x_q", "qwk_adjoint_r32_x_q",
    "qwk_adjoint_r64_x_q", "qwk_adjoint_rg1_x_q", "qwk_adjoint_rg2_x_q", "qwk_adjoint_rg4_x_q",
    "qwk_adjoint_rg8_x_q", "qwk_adjoint_r16w_x_q", "qwk_adjoint_r32w_x_q", "qwk_adjoint_r64w_x_q",
    "qwk_swap_real",
    "qwk_weight_real",  "qwk_grad_init_real", "qwk_gather_grad", "qwk_rot_table",
    "qwk_key_bits",     "qwk_radix_hist",   "qwk_radix_offsets", "qwk_radix_scatter",
    "qwk_split_amps"};
static_assert(sizeof(kNames) / sizeof(kNames[0]) == F_COUNT, "one kernel name per Fn");

// 0..3 for slmax = 1, 2, 4, 8
int width_index(int32_t slmax) { return slmax <= 1 ? 0 : slmax <= 2 ? 1 : slmax <= 4 ? 2 : 3; }

int log2_of(int32_t s) {
  int lg = 0;
  while ((1 << lg) < s) ++lg;
  return lg;
}

// Matrix::xcd for one launch of the one-pass step and adjoint kernels: the
// workgroups per XCD when the context asks for the XCD numbering (-1) and the
// grid is a multiple of 8, else 0 (the plain numbering).
int16_t xcd_blocks(const Matrix& m, int grid) {
  return m.xcd < 0 && grid % 8 == 0 && grid / 8 <= INT16_MAX ? int16_t(grid / 8) : int16_t(0);
}

Fn step_kernel(const StepArgs& a, int grid, int block) {
  const Matrix& m = a.m;
  const bool acc = a.yacc != nullptr;
  const int64_t work = m.waves + (int64_t(a.L.cnt) + kWave - 1) / kWave;
  const bool one_pass = m.full && a.mode == kStep && int64_t(grid) * (block / kWave) >= work;
  const bool wide = m.wide && m.suni >= 16;  // compile-time kernels with 16 lanes per row
  if (a.real) {  // the caller checked the conditions (launch_step re-checks them)
    const int f = m.suni > 0 && wide ? (m.angles ? F_STEP_TW16 : F_STEP_RW16) + log2_of(m.suni) - 4
                  : m.suni > 0       ? (m.angles ? F_STEP_T1 : F_STEP_R1) + log2_of(m.suni)
                                     : (m.angles ? F_STEP_TG1 : F_STEP_RG1) + width_index(m.slmax);
    return Fn(f + (acc ? int(F_REAL_COUNT_) : 0) + (a.q0 ? 2 * int(F_REAL_COUNT_) : 0) +
              (m.xcd > 0 ? 4 * int(F_REAL_COUNT_) : 0));
  }
  int f = F_STEP_S1 + width_index(m.slmax);
  if (m.vim) {
    f = (one_pass ? F_STEP_H1 : F_STEP_C1) + width_index(m.slmax);
    if (one_pass && m.suni > 0) f = wide ? F_STEP_KW16 + log2_of(m.suni) - 4 : F_STEP_K1 + log2_of(m.suni);
  } else if (m.angles) {
    f = (one_pass ? F_STEP_Y1 : F_STEP_X1) + width_index(m.slmax);
  } else if (one_pass) {
    f = F_STEP_G1 + width_index(m.slmax);
    if (m.suni > 0) f = wide ? F_STEP_FW16 + log2_of(m.suni) - 4 : F_STEP_F1 + log2_of(m.suni);
  }
  return Fn(f + (acc ? int(F_STEP_COUNT_) : 0));
}

constexpr int kMaxDevices = 64;

struct DeviceModule {
  hipModule_t mod;
  hipFunction_t fn[F_COUNT];
  void* scratch;  // this device's copy of the code object's `scratch` array
  size_t scratch_bytes;
  bool loaded;
};

DeviceModule g_dev[kMaxDevices];  // trivially destructible: nothing runs at exit
std::mutex g_mu;

hipError_t function(Fn f, hipFunction_t* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceModule& d = g_dev[dev];
  if (!d.loaded) {
    hipModule_t mod;
    e = hipModuleLoadData(&mod, qw_code_object);
    if (e != hipSuccess) return e;
    for (int i = 0; i < F_COUNT; ++i) {
      e = hipModuleGetFunction(&d.fn[i], mod, kNames[i]);
      if (e != hipSuccess) {
        (void)hipModuleUnload(mod);
        return e;
      }
    }
    // the address of this device's `scratch` array, looked up once per load
    // with the device current (a host-side name would not be a device address)
    // (a failed lookup leaves it unset: only qw_grad_noalloc needs it and
    // reports the error)
    void* sp = nullptr;
    size_t sb = 0;
    if (hipModuleGetGlobal(reinterpret_cast<hipDeviceptr_t*>(&sp), &sb, mod, "scratch") != hipSuccess ||
        sb < kScratchBytes) {
      sp = nullptr;
      sb = 0;
    }
    d.scratch = sp;
    d.scratch_bytes = sb;
    d.mod = mod;
    d.loaded = true;
  }
  *out = d.fn[f];
  return hipSuccess;
}

}  // namespace

hipError_t device_scratch(void** ptr, size_t* bytes) {
  hipFunction_t fn;
  hipError_t e = function(F_FILL, &fn);  // loads the module on this device if needed
  if (e != hipSuccess) return e;
  int dev = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_mu);
  *ptr = g_dev[dev].scratch;
  *bytes = g_dev[dev].scratch_bytes;
  return *ptr ? hipSuccess : hipErrorInvalidSymbol;
}

namespace {

hipError_t launch(Fn f, int grid, int block, hipStream_t stream, void** params) {
  hipFunction_t fn;
  hipError_t e = function(f, &fn);
  if (e != hipSuccess) return e;
  return hipModuleLaunchKernel(fn, unsigned(grid), 1, 1, unsigned(block), 1, 1, 0, stream, params, nullptr);
}

int clamp_grid(int64_t work, int64_t limit) {
  int64_t g = (work + 255) / 256;
  if (g < 1) g = 1;
  if (g > limit) g = limit;
  return int(g);
}

}  // namespace

hipError_t launch_step(const StepArgs& a, int grid, int block, hipStream_t stream) {
  if (block < kWave || block > kMaxBlock || block % kWave) return hipErrorInvalidValue;
  if (a.real && (a.mode != kStep || a.m.vim || a.L.cnt || !a.m.full ||
                 int64_t(grid) * (block / kWave) < a.m.waves))
    return hipErrorInvalidValue;  // the real-amplitude kernels are one-pass walk steps only
  StepArgs c = a;
  c.wpb = block / kWave;
  c.m.xcd = xcd_blocks(a.m, grid);
  if (c.m.xcd > 0 && a.real) c.wpb |= int32_t(c.m.xcd) << 8;  // the _x kernels' workgroups per XCD
  void* p[] = {&c};
  return launch(step_kernel(c, grid, block), grid, block, stream, p);
}

hipError_t launch_adjoint(const AdjArgs& a, int grid, int block, hipStream_t stream) {
  if (block < kWave || block > kMaxBlock || block % kWave) return hipErrorInvalidValue;
  // FP64 values only; complex values (vim) on the complex-plane kernels, with dvi
  if (a.m.angles || (a.m.vim != nullptr) != (a.dvi != nullptr) || (a.m.vim && a.real)) return hipErrorInvalidValue;
  AdjArgs c = a;
  c.wpb = block / kWave;
  c.m.xcd = xcd_blocks(a.m, grid);
  if (c.m.xcd > 0 && a.real) c.wpb |= int32_t(c.m.xcd) << 8;  // the _x kernels' workgroups per XCD
  if (!a.real) {
    c.real = 0;
    void* p[] = {&c};
    return launch(Fn(F_ADJOINT_S1 + width_index(a.m.slmax)), grid, block, stream, p);
  }
  // one pass over every wavefront, no lists (the caller checked; re-checked here)
  if (a.L.cnt || a.LL.cnt || !a.m.full || int64_t(grid) * (block / kWave) < a.m.waves) return hipErrorInvalidValue;
  const bool wide = a.m.wide && a.m.suni >= 16;
  const int f = a.m.suni > 0 && wide ? F_ADJ_RW16 + log2_of(a.m.suni) - 4
                : a.m.suni > 0       ? F_ADJ_R1 + log2_of(a.m.suni)
                                     : F_ADJ_RG1 + width_index(a.m.slmax);
  void* p[] = {&c};
  return launch(Fn(f + (a.q0 ? int(F_ADJ_COUNT_) : 0) + (c.m.xcd > 0 ? 2 * int(F_ADJ_COUNT_) : 0)), grid, block, stream,
                p);
}

hipError_t launch_rot_table(const Matrix& m, double* sfg, hipStream_t stream) {
  Matrix mm = m;
  void* p[] = {&mm, &sfg};
  return launch(F_ROT_TABLE, clamp_grid(m.items, 4096), 256, stream, p);
}

hipError_t launch_qbs_table(const Matrix& m, SlotRec* rec, uint32_t* slink, double* sval, hipStream_t stream) {
  Matrix mm = m;
  void* p[] = {&mm, &rec, &slink, &sval};
  return launch(F_QBS_TABLE, clamp_grid(m.items, 4096), 256, stream, p);
}

hipError_t launch_init(const Matrix& m, const double2* b, Slots out, double tau, hipStream_t stream) {
  Matrix mm = m;
  const double2* bb = b;
  double t = tau;
  void* p[] = {&mm, &bb, &out, &t};
  return launch(F_INIT, clamp_grid(m.items, 4096), 256, stream, p);
}

hipError_t launch_fill(void* ptr, int64_t bytes, hipStream_t stream) {
  int64_t n16 = bytes / 16;  // callers pass multiples of 16 bytes
  if (n16 <= 0) return hipSuccess;
  uint4* q = static_cast<uint4*>(ptr);
  void* p[] = {&q, &n16};
  return launch(F_FILL, clamp_grid(n16, 4096), 256, stream, p);
}

hipError_t launch_sum_counts(const unsigned long long* a, int64_t n, unsigned long long* out, hipStream_t stream) {
  void* p[] = {&a, &n, &out};
  return launch(F_SUM_COUNTS, kSumBlocks, 256, stream, p);
}

hipError_t launch_coef_window(const double* table, int64_t* base, double* window, int32_t count, int64_t set,
                              hipStream_t stream) {
  if (count < 0) return hipErrorInvalidValue;  // one wavefront fills the window, kWave entries at a time
  void* p[] = {&table, &base, &window, &count, &set};
  return launch(F_COEF_WINDOW, 1, kWave, stream, p);
}

hipError_t launch_to_real(const double2* src, double* dst, const double* val, int64_t n, hipStream_t stream) {
  void* p[] = {&src, &dst, &val, &n};
  return launch(F_TO_REAL, clamp_grid(n, 4096), 256, stream, p);
}

hipError_t launch_to_complex(const double* src, double2* dst, const double* val, int64_t n, hipStream_t stream) {
  void* p[] = {&src, &dst, &val, &n};
  return launch(F_TO_COMPLEX, clamp_grid(n, 4096), 256, stream, p);
}

hipError_t launch_measure(const Matrix& m, Slots st, List L, int32_t kind, double* partial, double* out, int grid,
                          hipStream_t stream) {
  Matrix mm = m;
  int32_t k = kind;
  if (kind <= 1 || kind == 4) {
    void* p[] = {&mm, &st, &L, &k, &partial};
    return launch(F_MEASURE, grid, 256, stream, p);
  }
  void* p[] = {&mm, &st, &L, &k, &out};
  return launch(F_MEASURE_ROWS, clamp_grid(m.rows + L.cnt, 4096), 256, stream, p);
}

hipError_t launch_export(const Matrix& m, Slots st, List L, uint64_t* keys, double2* amps, uint32_t* count,
                         uint32_t cap, hipStream_t stream) {
  Matrix mm = m;
  void* p[] = {&mm, &st, &L, &keys, &amps, &count, &cap};
  return launch(F_EXPORT, 1024, 256, stream, p);
}

hipError_t launch_key_bits(const uint64_t* keys, int64_t count, unsigned long long* bits, hipStream_t stream) {
  const uint64_t* k = keys;
  int64_t n = count;
  void* p[] = {&k, &n, &bits};
  return launch(F_KEY_BITS, clamp_grid(n, 1024), 256, stream, p);
}

hipError_t launch_radix_pass(const uint64_t* kin, const double2* vin, int64_t count, int shift, uint32_t* hist,
                             uint32_t* digit_base, uint64_t* kout, double2* vout, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  int64_t tiles = (count + kSortTile - 1) / kSortTile;
  if (tiles > int64_t(INT32_MAX)) return hipErrorInvalidValue;
  const uint64_t* ki = kin;
  const double2* vi = vin;
  int64_t n = count;
  int sh = shift;
  void* ph[] = {&ki, &n, &sh, &hist};
  hipError_t e = launch(F_RADIX_HIST, int(tiles), 256, stream, ph);
  if (e != hipSuccess) return e;
  void* po[] = {&hist, &tiles, &digit_base};
  e = launch(F_RADIX_OFFSETS, 1, 256, stream, po);
  if (e != hipSuccess) return e;
  const uint32_t* h = hist;
  const uint32_t* db = digit_base;
  void* ps[] = {&ki, &vi, &n, &sh, &h, &db, &kout, &vout};
  return launch(F_RADIX_SCATTER, int(tiles), 256, stream, ps);
}

hipError_t launch_split_amps(const double2* a, int64_t n, double* re, double* im, hipStream_t stream) {
  const double2* aa = a;
  int64_t nn = n;
  void* p[] = {&aa, &nn, &re, &im};
  return launch(F_SPLIT_AMPS, clamp_grid(n, 2048), 256, stream, p);
}

hipError_t launch_import(const Matrix& m, const uint64_t* keys, const double2* amps, int64_t n, Slots out, List L,
                         uint32_t* lcnt, hipStream_t stream) {
  Matrix mm = m;
  const uint64_t* k = keys;
  const double2* a = amps;
  int64_t cnt = n;
  void* p[] = {&mm, &k, &a, &cnt, &out, &L, &lcnt};
  return launch(F_IMPORT, clamp_grid(n, 2048), 256, stream, p);
}

hipError_t launch_weight(const Matrix& m, Slots in, List L, Slots out, List LL, const double* w, double* partial,
                         int grid, hipStream_t stream) {
  Matrix mm = m;
  const double* ww = w;
  void* p[] = {&mm, &in, &L, &out, &LL, &ww, &partial};
  return launch(F_WEIGHT, grid, 256, stream, p);
}

hipError_t launch_swap_real(const Matrix& m, Slots in, Slots out, unsigned long long* acc, hipStream_t stream) {
  Matrix mm = m;
  void* p[] = {&mm, &in, &out, &acc};
  return launch(F_SWAP_REAL, clamp_grid(m.items, 4096), 256, stream, p);
}

hipError_t launch_weight_real(const Matrix& m, Slots in, Slots out, const double* w, double* partial, int grid,
                              hipStream_t stream) {
  Matrix mm = m;
  const double* ww = w;
  void* p[] = {&mm, &in, &out, &ww, &partial};
  return launch(F_WEIGHT_REAL, grid, 256, stream, p);
}

hipError_t launch_grad_init_real(const Matrix& m, Slots lam, const double2* b, double* dv, double2* db,
                                 hipStream_t stream) {
  Matrix mm = m;
  const double2* bb = b;
  void* p[] = {&mm, &lam, &bb, &dv, &db};
  // one lane per row: 64-lane workgroups spread the rows over more CUs
  return launch(F_GRAD_INIT_REAL, clamp_grid(4 * m.rows, 16384), 64, stream, p);
}

hipError_t launch_gather_grad(const double* dv, const int32_t* home, int64_t nnz, const double2* db,
                              const int32_t* row, int64_t n, double* gv, double* br, double* bi,
                              const double* dvi, double* gvi, hipStream_t stream) {
  if ((dvi == nullptr) != (gvi == nullptr)) return hipErrorInvalidValue;
  void* p[] = {&dv, &home, &nnz, &db, &row, &n, &gv, &br, &bi, &dvi, &gvi};
  return launch(F_GATHER_GRAD, clamp_grid(nnz + n, 4096), 256, stream, p);
}

hipError_t launch_grad_init(const Matrix& m, Slots lam, const double2* b, double* dv, double2* db, double* dvi,
                            hipStream_t stream) {
  if (m.angles || (m.vim != nullptr) != (dvi != nullptr)) return hipErrorInvalidValue;
  Matrix mm = m;
  const double2* bb = b;
  void* p[] = {&mm, &lam, &bb, &dv, &db, &dvi};
  return launch(F_GRAD_INIT, clamp_grid(4 * m.rows, 16384), 64, stream, p);  // as launch_grad_init_real
}

}  // namespace qw

extern "C" void qw_shutdown(void) {
  try {  // no C++ exception leaves the library (std::mutex::lock may throw)
    std::lock_guard<std::mutex> lock(qw::g_mu);
    int cur = 0;
    const bool have_dev = hipGetDevice(&cur) == hipSuccess;
    for (int d = 0; d < qw::kMaxDevices; ++d) {
      if (!qw::g_dev[d].loaded) continue;
      if (hipSetDevice(d) == hipSuccess) (void)hipModuleUnload(qw::g_dev[d].mod);
      qw::g_dev[d].loaded = false;
    }
    if (have_dev) (void)hipSetDevice(cur);
  } catch (...) {
  }
}
