// HIP kernels of the quantum-walk library, written for gfx950 (CDNA4, wave64).
//
// Walk step (Alg. 6 of arXiv:2303.06890, W = S T~ P T~^dagger).  With
// T~ = O_s' R H (Alg. 5: the QRAM read of a_{j,l}, the rotation and the
// uncompute collapse to a rotation controlled by the slot) the middle part
// R H P H R^dagger, seen after O_s'^-1, is
//   2 |phi_j><phi_j| - 1  on the 2s amplitudes (l, b2) of a group
//                         (j_c = 0, j, b1 = 0, z = 0),
//   -1                    on every other branch,
// with phi_j(l, 0) = f_{jl}/sqrt(s), phi_j(l, 1) = g_{jl}/sqrt(s) (P of
// Eq. "impl" flips every branch but |j~>).  O_s' and S are bijections of the
// keys, so the only interference in a step is one reduction per group j.
//
// The members of group j are the keys K(q, b2) = (0, j, 0, 0, col[q], b2) of
// the ELL slots q = (j, l) of row j; after O_s' and S the reflected outputs
// are S K(q, b2) = (0, col[q], b2, 0, j, 0).  S K(q, 1) is never a group
// member (b1 = 1); S K(q, 0) is the member K(q', 0) of slot
// q' = (col[q], rev[q]) when j is in row col[q] (rev = the quantum binary
// search of j in that row, tabulated once per matrix), and not a member
// otherwise.  One step later every S K(q, b2) that is not a member is mapped
// back to K(q, b2) (by -S).  So every branch reachable from T~|b~> has a
// fixed address, in four planes indexed by the slot's home
// h = base + l*N + j (slot-position-major, so that the slots of one position
// l of consecutive rows are contiguous):
//   R0[h], R1[h]: K(q, 0), K(q, 1)         (group members)
//   Q1[h]:        S K(q, 1)
//   Q0[h]:        S K(q, 0) when rev[q] < 0 (never written otherwise)
// One launch per step reads the planes of a row's slots, reduces the group
// across the lanes of the row, and writes each output to its address for the
// next step:
//   R0, R1 -> reflection -> Q1_out[h] and R0_out[h'] (or Q0_out[h])
//   Q1, Q0 -> negation   -> R1_out[h], R0_out[h]
// R1_out = -Q1_in is never copied: a state keeps three planes per parity
// buffer, and its R1 is the other buffer's Q1 plane times a sign (+-1) that
// the state carries (a walk step leaves -1, the swap +1).  So a step writes
// three planes (R0, Q1 and the fillers' Q0) and reads R1 from the plane it
// then overwrites with Q1.
// Every output address receives exactly one write per step (0 when pruned;
// the cells that provably stay 0, of slots of value 0, are skipped), so there
// is no atomic, no compaction and no clearing pass; the result is independent
// of scheduling.  For matrices whose rows share their offset
// pattern (band and circulant-offset matrices) the partner writes R0_out[h']
// of a wavefront are contiguous too.  Branches outside that span (only from
// raw starts or imports) sit in a list that W maps in place to -S(key).
#include "qw_internal.h"

#include <hip/hip_runtime.h>

// Device memory of qw_grad_noalloc: a fixed array of the code object, one
// per device that loads it, held from the load to qw_shutdown.  No kernel
// names it.  The host looks its address up on each device's module
// (hipModuleGetGlobal, which needs an exported name; the `used` attribute
// keeps the unreferenced array in the code object) and passes it to the
// kernels as an ordinary pointer.
// (A braced linkage block: `extern "C"` before a lone declaration would
// make it a declaration, not a definition.)
extern "C" {
__device__ __attribute__((used)) __align__(256) unsigned char scratch[qw::kScratchBytes];
}

namespace qw {

// ----------------------------------------------------------------- helpers

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cneg(double2 a) { return make_double2(-a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double t) { return make_double2(a.x * t, a.y * t); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 cjmul(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double norm2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ bool kept(double2 v, double tau) { return fabs(v.x) > tau || fabs(v.y) > tau; }
__device__ __forceinline__ bool nonzero(double2 v) { return v.x != 0.0 || v.y != 0.0; }
__device__ __forceinline__ double2 zero2() { return make_double2(0.0, 0.0); }
// value, or exact 0 when it falls to the pruning threshold
__device__ __forceinline__ double2 prune(double2 v, double tau, unsigned& cnt) {
  if (kept(v, tau)) {
    ++cnt;
    return v;
  }
  return zero2();
}

// Rotation amplitudes of Sec. IV (footnote on negative elements):
// f = sqrt(a) for a >= 0, +-i sqrt|a| (+ when row j <= column k) for a < 0,
// g = sqrt(1 - |a|).
struct Rot {
  double2 f;
  double g;
};
// `upper`: row j <= column k.
__device__ __forceinline__ Rot rot_real(double a, bool upper) {
  Rot r;
  const double q = sqrt(fabs(a));  // no divergent branch
  r.f = a >= 0.0 ? make_double2(q, 0.0) : make_double2(0.0, upper ? q : -q);
  r.g = sqrt(1.0 - fabs(a));
  return r;
}
__device__ __forceinline__ Rot rotation(double a, int j, int k) { return rot_real(a, j <= k); }
// A complex value a + i b held by row j (the row holds A*_{jk} of a Hermitian
// matrix): off the real axis f = the principal sqrt(a + i b), so that
// sqrt(A*_{jk}) of psi_j appears as in Sec. IV, and g = sqrt(1 - |a + i b|);
// on the axis the real rule above.
__device__ __forceinline__ Rot rot_cplx(double a, double b, bool upper) {
  if (b == 0.0) return rot_real(a, upper);
  Rot r;
  const double m = hypot(a, b);
  const double t = sqrt(0.5 * (m + fabs(a)));  // > 0 since b != 0
  r.f = a >= 0.0 ? make_double2(t, 0.5 * b / t) : make_double2(0.5 * fabs(b) / t, copysign(t, b));
  r.g = sqrt(1.0 - m);
  return r;
}
__device__ __forceinline__ Rot rotation(double a, double b, int j, int k) { return rot_cplx(a, b, j <= k); }
// Fixed-point data: the host has turned each value into the signed angle y
// of its rotation (units of pi); f = sin(pi |y|), with the +-i rule of the
// real case when y < 0, and g = cos(pi y).  sincospi is exact at y = 0.
__device__ __forceinline__ Rot rot_angle(double y, bool upper) {
  double sv, cv;
  sincospi(fabs(y), &sv, &cv);
  Rot r;
  r.f = !signbit(y) ? make_double2(sv, 0.0) : make_double2(0.0, upper ? sv : -sv);
  r.g = cv;
  return r;
}
__device__ __forceinline__ Rot rotation_angle(double y, int j, int k) { return rot_angle(y, j <= k); }
// Rotation of slot home h whatever the matrix holds (outside the step kernels).
__device__ __forceinline__ Rot rotation_of(const Matrix& m, double val, int64_t h, int j, int k) {
  if (m.angles) return rotation_angle(val, j, k);
  return rotation(val, m.vim ? m.vim[h] : 0.0, j, k);
}
// d f/da and d g/da (not finite at a = 0 and |a| = 1).
__device__ __forceinline__ Rot rotation_deriv(double a, int j, int k) {
  Rot d;
  const double q = 0.5 / sqrt(fabs(a));  // +inf at a = 0
  d.f = a > 0.0 ? make_double2(q, 0.0)
                : (a < 0.0 ? make_double2(0.0, j <= k ? -q : q) : make_double2(__builtin_inf(), 0.0));
  const double sg = a > 0.0 ? 1.0 : (a < 0.0 ? -1.0 : 0.0);
  d.g = -sg * 0.5 / sqrt(1.0 - fabs(a));
  return d;
}
// The same for a complex value a + i b (rot_cplx), with respect to a
// (im = false) or to b (im = true).  Off the axis f = sqrt(a + i b) is
// holomorphic: df/da = 1/(2f), df/db = i/(2f); |v| = hypot(a, b) gives
// dg/da = -a/(2|v|g), dg/db = -b/(2|v|g).  On the axis rot_cplx takes the
// real rule: with respect to a that is rotation_deriv; with respect to b the
// principal root is analytic for a > 0 (df/db = i/(2 sqrt a), dg/db = 0) and
// has no derivative for a <= 0 (the +-i rule sits on its cut): NaN.
__device__ __forceinline__ Rot rotation_deriv_c(double a, double b, int j, int k, bool im) {
  if (b == 0.0) {
    if (!im) return rotation_deriv(a, j, k);
    Rot d;
    const double q = a > 0.0 ? 0.5 / sqrt(a) : __builtin_nan("");
    d.f = make_double2(a > 0.0 ? 0.0 : q, q);
    d.g = a > 0.0 ? 0.0 : q;
    return d;
  }
  const Rot r = rot_cplx(a, b, true);  // off the axis the row order does not matter
  const double m = hypot(a, b);
  // 1/(2f) = conj(f) / (2|f|^2), |f|^2 = |v|
  const double2 h = make_double2(0.5 * r.f.x / m, -0.5 * r.f.y / m);
  Rot d;
  d.f = im ? make_double2(-h.y, h.x) : h;
  d.g = -0.5 * (im ? b : a) / (m * r.g);
  return d;
}
// The rotation of a + i b and its derivatives by a and by b together
// (rot_cplx, rotation_deriv_c): off the axis one hypot, the two square roots
// of the rotation and two reciprocals (1/|v|, 1/g) serve all three, which
// the reverse step needs for every slot.
__device__ __forceinline__ void rot_and_derivs(double a, double b, int j, int k, Rot& r, Rot& da, Rot& db) {
  if (b == 0.0) {
    r = rot_real(a, j <= k);
    da = rotation_deriv(a, j, k);
    db = rotation_deriv_c(a, 0.0, j, k, true);
    return;
  }
  const double m = hypot(a, b);
  const double t = sqrt(0.5 * (m + fabs(a)));  // > 0 since b != 0
  r.f = a >= 0.0 ? make_double2(t, 0.5 * b / t) : make_double2(0.5 * fabs(b) / t, copysign(t, b));
  r.g = sqrt(1.0 - m);
  const double im = 1.0 / m;
  const double2 h = make_double2(0.5 * r.f.x * im, -0.5 * r.f.y * im);  // 1/(2f) = conj(f) / (2|v|)
  const double kg = -0.5 * im / r.g;
  da.f = h;
  da.g = a * kg;
  db.f = make_double2(-h.y, h.x);
  db.g = b * kg;
}
// conj(f) x0 + g x1: the component of an amplitude pair along sqrt(s) phi
__device__ __forceinline__ double2 along(const Rot& r, double2 x0, double2 x1) {
  return cadd(cjmul(r.f, x0), cscale(x1, r.g));
}

// Quantum binary search (Definition of QBS, Sec. III.A) as a per-branch
// function: position of `target` in the sorted row of length s (a power of
// two), log2(s) probes plus the value at position 0.
__device__ __forceinline__ bool qbs(const int32_t* __restrict__ row, int s, int target, int& pos) {
  int p = 0;
  int vp = row[0];
  for (int step = s >> 1; step > 0; step >>= 1) {
    const int v = row[p + step];
    if (v <= target) {
      p += step;
      vp = v;
    }
  }
  pos = p;
  return vp == target;
}

// Value of a double in the lane selected by a DPP pattern (within rows of 16).
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false),
                          __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false));
}
// v plus its value in lane ^ 16 (lane ^ 32): gfx950's cross-row swaps
// (v_permlane16_swap, v_permlane32_swap) exchange the two halves of each
// pair of 16-lane rows (of the wavefront) in the vector ALU, where a lane
// shuffle is an LDS round trip.  Both lanes of a pair add the same two
// values in the same order, so their sums are bitwise identical.
__device__ __forceinline__ double swap_add_16(double v) {
  const unsigned lo = __double2loint(v), hi = __double2hiint(v);
  const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
}
__device__ __forceinline__ double swap_add_32(double v) {
  const unsigned lo = __double2loint(v), hi = __double2hiint(v);
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
}
// Sum over the lanes that hold one row in the step kernels: lanes
// jj + h * 2^rpw_log, h < 2^(6 - rpw_log), rpw_log >= 2.  Within a row of
// 16 lanes: + lane ^ 8 (a rotation by 8), then, for 16 lanes per row, + the
// lane 4 further on (its sum of {l + 4, l + 12} against {l, l + 8}).  Across
// rows: the swaps above when a lane holds at most two slots; with more, the
// vector ALU is busy with the slots' square roots, and lane shuffles through
// the LDS, another unit, are faster (per step: shapes B and C 6 % and 5 %
// faster with the swaps, G(16384, 8) 1.5 %, the batch 1 %; shape E, eight
// slots per lane, 2 % slower).  Every lane of a row ends with the
// bitwise-identical sum (each stage adds a commuted pair).
template <int SLM>
__device__ __forceinline__ double row_sum_r(double v, int rpw_log) {
  if (rpw_log <= 3) v += dpp<0x128>(v);
  if (rpw_log <= 2) v += dpp<0x124>(v);
  if constexpr (SLM <= 2) {
    if (rpw_log <= 4) v = swap_add_16(v);
    if (rpw_log <= 5) v = swap_add_32(v);
  } else {
    if (rpw_log <= 4) v += __shfl_xor(v, 16);
    if (rpw_log <= 5) v += __shfl_xor(v, 32);
  }
  return v;
}
template <int SLM>
__device__ __forceinline__ double2 row_sum(double2 v, int rpw_log) {
  return make_double2(row_sum_r<SLM>(v.x, rpw_log), row_sum_r<SLM>(v.y, rpw_log));
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// 2/s of the reflection 2 |phi><phi| - 1 (phi carries 1/sqrt(s) per entry):
// a constant for a compile-time s, else one ldexp (s = 2^hbits, so both are
// exact); a division here sat on every wavefront's path after the row sum.
template <int S>
__device__ __forceinline__ double two_over_s(const Inst& I) {
  return S ? 2.0 / double(S) : ldexp(2.0, -I.hbits);
}

// Read-only loads from a wavefront-uniform address, through the scalar cache
// (the constant address space).
typedef const __attribute__((address_space(4))) Inst* ConstInstPtr;
__device__ __forceinline__ int32_t uload(const int32_t* p) {
  return *(const __attribute__((address_space(4))) int32_t*)p;
}
__device__ __forceinline__ Inst uload(const Inst* p) {
  const ConstInstPtr c = (ConstInstPtr)p;
  Inst I;
  I.item_base = c->item_base;
  I.jbase = c->jbase;
  I.wave_base = c->wave_base;
  I.N = c->N;
  I.s = c->s;
  I.hbits = c->hbits;
  I.nlog = c->nlog;
  I.lpr_log = c->lpr_log;
  I.sl = c->sl;
  I.inv_sqrt_s = c->inv_sqrt_s;
  return I;
}

// Instance whose range starts at or before x (ranges ordered by field F);
// x may differ between lanes.
template <int64_t Inst::*F>
__device__ __forceinline__ int find_inst(const Matrix& m, int64_t x) {
  int lo = 0, hi = m.ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (m.inst[mid].*F <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}
// The same for a wavefront-uniform x, with scalar loads.
template <int64_t Inst::*F>
__device__ __forceinline__ int find_inst_uniform(const Matrix& m, int64_t x) {
  int lo = 0, hi = m.ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (((ConstInstPtr)(m.inst + mid))->*F <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}
// Instance record by wavefront-uniform index.
__device__ __forceinline__ Inst inst_uniform(const Matrix& m, int i) {
  Inst I;
  if (m.ninst == 1)
    I = m.inst0;
  else
    I = uload(m.inst + i);
  return I;
}

__device__ __forceinline__ uint64_t swap_halves(uint64_t key, int n) {
  const int h = 2 * n + 1;
  const uint64_t hm = (uint64_t(1) << h) - 1;
  const uint64_t lo = key & hm, hi = (key >> h) & hm, top = key >> (2 * h);
  return (top << (2 * h)) | (lo << h) | hi;
}

// K(q, b2) = (0, j, 0, 0, col, b2) of instance `inst`.
__device__ __forceinline__ uint64_t member_key(uint64_t inst, int n, int j, int col, int b2) {
  return (inst << (4 * n + 2)) | (uint64_t(j) << (2 * n + 2)) | (uint64_t(col) << 1) | uint64_t(b2);
}
// S K(q, b2) = (0, col, b2, 0, j, 0).
__device__ __forceinline__ uint64_t swapped_key(uint64_t inst, int n, int j, int col, int b2) {
  return (inst << (4 * n + 2)) | (uint64_t(col) << (2 * n + 2)) | (uint64_t(b2) << (2 * n + 1)) |
         (uint64_t(j) << 1);
}

// Home of slot (j, l): the state planes and the slot records; the ELL arrays
// col/val are row-major (base + j*s + l) for the binary searches.
__device__ __forceinline__ int64_t home(const Inst& I, int j, int l) {
  return I.item_base + (int64_t(l) << I.nlog) + j;
}

// A lane of a pass over homes.  `first` is the first home of the lane's
// wavefront: instances start at multiples of 64, so a wavefront never
// straddles two and its instance is looked up once, uniformly.
struct Home {
  Inst I;
  int inst;
  int j, l;
  bool live;
};
__device__ __forceinline__ Home home_item(const Matrix& m, int64_t it, int64_t first) {
  Home x;
  x.inst = m.ninst == 1 ? 0 : find_inst_uniform<&Inst::item_base>(m, uniform(int(first >> 6)) * int64_t(64));
  x.I = inst_uniform(m, x.inst);
  const int64_t local = it - x.I.item_base;
  x.live = local < (int64_t(x.I.N) << x.I.hbits);
  x.l = int(local >> x.I.nlog);
  x.j = int(local & (x.I.N - 1));
  return x;
}

// A lane of a pass over rows (one lane per row j of every instance).
struct Row {
  Inst I;
  int inst;
  int j;
};
__device__ __forceinline__ Row row_item(const Matrix& m, int64_t r) {
  Row x;
  x.inst = m.ninst == 1 ? 0 : find_inst<&Inst::jbase>(m, r);
  x.I = m.inst[x.inst];
  x.j = int(r - x.I.jbase);
  return x;
}

// Lane mapping of the step kernels for s = S: min(S, 8) lanes share a row,
// each holding S / min(S, 8) slots; W (Matrix::wide): 16 lanes for S >= 16.
template <int S, int W = 0>
struct Shape {
  static constexpr int lpr_log = W && S >= 16 ? 4 : S >= 8 ? 3 : (S == 4 ? 2 : (S == 2 ? 1 : 0));
  static constexpr int rpw_log = 6 - lpr_log;
  static constexpr int sl = S >> lpr_log;
};

// A lane of the step kernels: wavefront w of the instance covers rows
// [w * 2^rpw_log, (w + 1) * 2^rpw_log); lane = h * 2^rpw_log + jj holds slots
// l = h * sl + i (i < sl) of row w * 2^rpw_log + jj.  S != 0: every instance
// has s = S (the mapping is known at compile time).
struct Lanes {
  Inst I;
  int inst;
  int j, h, rpw_log;
  bool live;
};
template <int S, bool FULL = false, int W = 0>
__device__ __forceinline__ Lanes lanes_of(const Matrix& m, int64_t w, int lane) {
  Lanes x;
  x.inst = m.ninst == 1 ? 0 : uload(m.wave_inst + w);
  x.I = inst_uniform(m, x.inst);
  x.rpw_log = S ? Shape<S, W>::rpw_log : 6 - x.I.lpr_log;
  x.h = lane >> x.rpw_log;
  const int64_t j = ((w - x.I.wave_base) << x.rpw_log) + (lane & ((1 << x.rpw_log) - 1));
  x.live = FULL || j < x.I.N;  // FULL: every N is a multiple of 2^rpw_log
  x.j = x.live ? int(j) : 0;   // rows past N (instances with N < 2^rpw_log) read row 0 and write nothing
  return x;
}

// Sum of a per-lane count over the wavefront, bit plane by bit plane with
// ballots and population counts (scalar work), not with a chain of lane
// shuffles: it sits on the path to the end of every wavefront.
__device__ __forceinline__ unsigned long long wave_sum(unsigned cnt) {
  unsigned long long v = 0;
  for (int b = 0; b < 32; ++b) {
    v += static_cast<unsigned long long>(__popcll(__ballot((cnt >> b) & 1u))) << b;
    if (__ballot((cnt >> b) > 1u) == 0) break;  // no higher bit set in any lane
  }
  return v;
}
// The same for counts below 2^BITS: one ballot per bit and no branch (the
// loop's early exit cost 0.09 us per launch at 16384 x 8).
template <int BITS>
__device__ __forceinline__ unsigned long long wave_sum_bits(unsigned cnt) {
  unsigned long long v = 0;
#pragma unroll
  for (int b = 0; b < BITS; ++b) v += static_cast<unsigned long long>(__popcll(__ballot((cnt >> b) & 1u))) << b;
  return v;
}
// Bits of a one-pass lane's count: at most 4 per slot (a kept Q1 output
// twice, then R0, or Q0 and R0), SLM slots.
template <int SLM>
struct CountBits {
  static constexpr int value = SLM == 1 ? 3 : SLM == 2 ? 4 : SLM == 4 ? 5 : 6;
};
// The running count of this wavefront in the step and adjoint kernels
// (kMaxWaves counters).
// Workgroups are dealt to the eight XCDs in turn, so the counters are grouped
// by XCD: the 16 counters of a cache line belong to wavefronts of one XCD,
// and a line is never written from two XCDs' caches in one launch.  Each
// counter has one writer, so a plain load at the start and a store at the
// end replace an atomic (the count store ends the wavefront's work; on a
// shared line it cost 0.17 us per launch at 16384 x 8).
// Row block of workgroup p in the one-pass step and adjoint kernels' _x forms.
// Workgroups are dealt to the eight XCDs in turn (workgroup p runs on XCD
// p % 8), each with its own L2.  Neighbouring row blocks share cache lines of
// the 4- and 8-byte planes (a 128-byte line of the link plane spans 32 rows),
// so the _x forms renumber the blocks to keep neighbours on one XCD: with xb =
// G / 8 workgroups per XCD (G a multiple of 8), workgroup p takes block
// (p % 8) * xb + p / 8.  A tuning choice: which workgroup runs which rows
// changes, nothing else.  The launcher passes xb in bits 8 and up of
// StepArgs::wpb / AdjArgs::wpb, the argument the prologue loads first anyway:
// a separate argument, or the grid read from the dispatch packet, put one
// more scalar load ahead of the data (2.52 against 2.47 us per step at
// 16384 x 8).
__device__ __forceinline__ int64_t xcd_row_block(int64_t p, int64_t xb) { return (p & 7) * xb + (p >> 3); }

__device__ __forceinline__ int64_t wave_counter(int64_t wpb) {
  return int64_t(blockIdx.x & 7) * (kMaxWaves / 8) + int64_t(blockIdx.x >> 3) * wpb + (threadIdx.x >> 6);
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < int(blockDim.x >> 6); ++i) t += sh[i];
  return t;
}

// Logical R1 amplitude of a home (the plane holds it times r1s = +-1).
__device__ __forceinline__ double2 r1_of(const Slots& st, int64_t h) { return cscale(st.R1[h], st.r1s); }

// Outputs of one slot for the next step (step and adjoint kernels).
// o0, o1: reflected (or swapped) group amplitudes of K(q, b2) before S; o1
// goes to Q1 at h, o0 to R0 at the partner's home (or, without a partner, to
// Q0 at h, with R0 at h <- Q0_in, negated when `neg`).  Q1_in becomes the
// next R1 (negated by a walk step, not by the swap) without being moved or
// read: the input's Q1 plane is the output's R1 storage, and the sign goes
// with the state.  out.Q1 is in.R1's plane: each lane reads its R1 input
// before it writes its Q1 output at the same home.
// Counts: every kept output once, and a kept Q1 output once more for the R1
// branch it becomes one launch later; the host corrects the sum by the Q1
// branches of the present state.  `zero`: a slot of value 0 in a state whose
// R0 and Q0 cells of such slots are 0 (StepArgs::zskip): o0 is then 0 and
// lands in such a cell, so the b2 = 0 path is skipped.
__device__ __forceinline__ void write_slot(const Slots& in, const Slots& out, int64_t base, int64_t h, int part,
                                           double2 o0, double2 o1, bool neg, double tau, unsigned& cnt,
                                           bool zero = false) {
  unsigned q1 = 0;
  out.Q1[h] = prune(o1, tau, q1);
  cnt += 2 * q1;
  if (zero) return;
  if (part >= 0) {
    out.R0[base + part] = prune(o0, tau, cnt);
  } else {
    const double2 y0 = in.Q0[h];
    out.Q0[h] = prune(o0, tau, cnt);
    out.R0[h] = prune(neg ? cneg(y0) : y0, tau, cnt);
  }
}

// In-place image of a list entry: W maps it to -S(key), S to S(key).
__device__ __forceinline__ unsigned list_entry(const List& L, int64_t e, int n, bool neg) {
  if (e >= int64_t(L.cnt)) return 0;
  double2 v = L.amp[e];
  if (neg) v = cneg(v);
  L.amp[e] = v;
  L.key[e] = swap_halves(L.key[e], n);
  return nonzero(v);
}

// ----------------------------------------------------------------- walk step

// The step kernels' record of slot home h, decoded.
struct StepSlot {
  int part;    // partner's home relative to the instance base, or -1
  bool upper;  // row j <= column col[q]
  double val;
};
__device__ __forceinline__ StepSlot step_rec(const Matrix& m, int64_t h) {
  const uint32_t link = m.slink[h];
  StepSlot t;
  t.val = m.sval[h];
  t.part = int(link & 0x7fffffffu) - 1;
  t.upper = (link >> 31) == 0u;
  return t;
}

// One wavefront of the step: up to SLM slots per lane, held in registers.
// The data loads do not depend on each other or on the instance record
// beyond its base, so they are issued together.  FAST: walk step (not the
// swap) and every row of every wavefront exists.
template <bool ACC, int SLM, int S, bool FAST, int ENC, int W = 0>
__device__ __forceinline__ unsigned step_wave(const StepArgs& a, int64_t w, int lane, double coef) {
  const Lanes x = lanes_of<S, FAST, W>(a.m, w, lane);
  const int sl = S ? Shape<S, W>::sl : (SLM == 1 ? 1 : x.I.sl);
  const int64_t base = x.I.item_base;
  int64_t h[SLM];
  StepSlot rc[SLM];
  double2 x0[SLM], x1[SLM];
  double vi[SLM];
  bool zero[SLM];
  Rot r[SLM];
  // Complex values, one s, at most two slots per lane: the rotation comes
  // from the table (Matrix::sfg, four doubles per slot) instead of the two
  // value planes and the principal square root (as the real kernels'
  // rotation table does, for the same reason: these steps are bound by
  // their chain of dependent operations).
  constexpr bool kTab = ENC == kEncComplex && S != 0 && SLM <= 2;
  double2 tf[SLM], tg[SLM];
#pragma unroll
  for (int i = 0; i < SLM; ++i) {
    if (i < sl) {
      h[i] = base + (int64_t(x.h * sl + i) << x.I.nlog) + x.j;
      if constexpr (kTab) {
        const uint32_t link = a.m.slink[h[i]];
        rc[i].part = int(link & 0x7fffffffu) - 1;  // as step_rec
        rc[i].upper = (link >> 31) == 0u;
        rc[i].val = 0.0;  // not read: the table holds the rotation
        vi[i] = 0.0;
        const double2* t = reinterpret_cast<const double2*>(a.m.sfg) + 2 * h[i];
        tf[i] = t[0];
        tg[i] = t[1];
      } else {
        rc[i] = step_rec(a.m, h[i]);
        if (ENC == kEncComplex) vi[i] = a.m.vim[h[i]];
      }
      x1[i] = r1_of(a.in, h[i]);
      // slots of value 0 (fillers): R0 stays 0 when the state allows it
      zero[i] = S == 0 && a.zskip && rc[i].val == 0.0 && (ENC != kEncComplex || vi[i] == 0.0);
      x0[i] = zero[i] ? zero2() : a.in.R0[h[i]];
    }
  }
  const bool step = FAST || a.mode == kStep;
  double2 c = zero2();
#pragma unroll
  for (int i = 0; i < SLM; ++i) {
    if (i < sl) {
      if constexpr (kTab) {
        r[i].f = tf[i];
        r[i].g = tg[i].x;
      } else {
        r[i] = ENC == kEncComplex ? rot_cplx(rc[i].val, vi[i], rc[i].upper)
               : ENC == kEncAngle ? rot_angle(rc[i].val, rc[i].upper)
                                  : rot_real(rc[i].val, rc[i].upper);
      }
      c = cadd(c, along(r[i], x0[i], x1[i]));
    }
  }
  if (step) c = row_sum<SLM>(c, x.rpw_log);
  if (ACC && x.live && x.h == 0) {
    double2 yv = a.yacc[x.I.jbase + x.j];
    yv.x += coef * (c.x * x.I.inv_sqrt_s);
    yv.y += coef * (c.y * x.I.inv_sqrt_s);
    a.yacc[x.I.jbase + x.j] = yv;
  }
  if (!x.live) return 0;
  const double2 tc = cscale(c, two_over_s<S>(x.I));
  unsigned cnt = 0;
#pragma unroll
  for (int i = 0; i < SLM; ++i) {
    if (i < sl) {
      double2 o0 = x0[i], o1 = x1[i];
      if (step) {
        o0 = csub(cmul(tc, r[i].f), x0[i]);
        o1 = csub(cscale(tc, r[i].g), x1[i]);
      }
      write_slot(a.in, a.out, base, h[i], rc[i].part, o0, o1, step, a.tau, cnt, zero[i]);
    }
  }
  return cnt;
}

// SLM: slots per lane held in registers; S: s of every instance, or 0 (read
// per instance, slots per lane <= SLM).  FAST: one pass (the grid covers
// every wavefront and the list), walk step only, every row exists.
template <bool ACC, int SLM, int S, bool FAST, int ENC, int W = 0>
__device__ __forceinline__ void step_body(const StepArgs& a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wpb = a.wpb;  // a kernel argument: reading the workgroup size costs a vector load
  const int64_t wid = int64_t(blockIdx.x) * wpb + (threadIdx.x >> 6);  // this wavefront's index
  const double coef = ACC ? *a.coef : 0.0;  // no dependent load: the pointer is this launch's
  const int64_t cidx = wave_counter(wpb);
  const bool counting = a.acc != nullptr;  // the solver's private walk keeps no counts
  const unsigned long long prev = counting ? a.acc[cidx] : 0ull;
  unsigned cnt = 0;
  if (FAST) {
    const int64_t w = uniform(int(wid));
    // the arguments in one scalar-load round trip, as in step_body_real
    asm volatile("" ::"s"(a.m.inst0.item_base), "s"(a.m.inst0.nlog), "s"(a.m.slink), "s"(a.m.sval), "s"(a.in.R0),
                 "s"(a.in.R1), "s"(a.out.R0), "s"(a.out.Q1), "s"(a.in.r1s), "s"(a.tau), "s"(a.m.vim));
    asm volatile("" ::"s"(a.m.ninst), "s"(a.m.inst0.wave_base), "s"(a.m.inst0.s), "s"(a.m.inst0.N), "s"(a.in.Q0),
                 "s"(a.out.Q0), "s"(a.m.inst0.inv_sqrt_s), "s"(a.m.inst0.jbase), "s"(a.m.inst), "s"(a.m.wave_inst));
    if (w < a.m.waves)
      cnt = step_wave<ACC, SLM, S, true, ENC, W>(a, w, lane, coef);
    else
      cnt = list_entry(a.L, (w - a.m.waves) * kWave + lane, a.m.nbits, true);
  } else {
    const int64_t total = a.m.waves + (int64_t(a.L.cnt) + kWave - 1) / kWave;
    const int64_t wstride = int64_t(gridDim.x) * wpb;
    for (int64_t w = uniform(int(wid)); w < total; w += wstride) {
      if (w < a.m.waves)
        cnt += step_wave<ACC, SLM, S, false, ENC>(a, w, lane, coef);
      else
        cnt += list_entry(a.L, (w - a.m.waves) * kWave + lane, a.m.nbits, a.mode == kStep);
    }
  }
  if (counting) {
    const unsigned long long v = FAST ? wave_sum_bits<CountBits<SLM>::value>(cnt) : wave_sum(cnt);
    if (lane == 0) a.acc[cidx] = prev + v;
  }
}

}  // namespace qw

// qwk_step_sN: any s per instance, up to N slots per lane (s <= 8N), any
// launch shape, walk step or swap; qwk_step_gN: the same s per instance, but
// every instance has at least one wavefront of rows, one pass, walk step;
// qwk_step_fS: as gN with s = S for every instance; qwk_step_cN: as sN for a
// complex Hermitian matrix; qwk_step_xN: as sN for fixed-point data;
// qwk_step_hN and qwk_step_yN: as gN for those two; qwk_step_kS: as fS for
// a complex Hermitian matrix.
#define QW_STEP_KERNEL(NAME, SLM, S, FAST, ENC)                                                    \
  extern "C" __global__ void __launch_bounds__(256) NAME(qw::StepArgs a) {                         \
    qw::step_body<false, SLM, S, FAST, ENC>(a);                                                     \
  }                                                                                                 \
  extern "C" __global__ void __launch_bounds__(256) NAME##_acc(qw::StepArgs a) {                   \
    qw::step_body<true, SLM, S, FAST, ENC>(a);                                                      \
  }
// The one-pass compile-time kernels with 16 lanes per row (Matrix::wide).
#define QW_STEP_KERNEL_W(NAME, SLM, S, ENC)                                                        \
  extern "C" __global__ void __launch_bounds__(256) NAME(qw::StepArgs a) {                         \
    qw::step_body<false, SLM, S, true, ENC, 1>(a);                                                  \
  }                                                                                                 \
  extern "C" __global__ void __launch_bounds__(256) NAME##_acc(qw::StepArgs a) {                   \
    qw::step_body<true, SLM, S, true, ENC, 1>(a);                                                   \
  }
QW_STEP_KERNEL(qwk_step_s1, 1, 0, false, qw::kEncReal)
QW_STEP_KERNEL(qwk_step_s2, 2, 0, false, qw::kEncReal)
QW_STEP_KERNEL(qwk_step_s4, 4, 0, false, qw::kEncReal)
QW_STEP_KERNEL(qwk_step_s8, 8, 0, false, qw::kEncReal)
QW_STEP_KERNEL(qwk_step_g1, 1, 0, true, qw::kEncReal)
QW_STEP_KERNEL(qwk_step_g2, 2, 0, true, qw::kEncReal)
QW_STEP_KERNEL(qwk_step_g4, 4, 0, true, qw::kEncReal)
QW_STEP_KERNEL(qwk_step_g8, 8, 0, true, qw::kEncReal)
QW_STEP_KERNEL(qwk_step_f1, 1, 1, true, qw::kEncReal)
QW_STEP_KERNEL(qwk_step_f2, 1, 2, true, qw::kEncReal)
QW_STEP_KERNEL(qwk_step_f4, 1, 4, true, qw::kEncReal)
QW_STEP_KERNEL(qwk_step_f8, 1, 8, true, qw::kEncReal)
QW_STEP_KERNEL(qwk_step_f16, 2, 16, true, qw::kEncReal)
QW_STEP_KERNEL(qwk_step_f32, 4, 32, true, qw::kEncReal)
QW_STEP_KERNEL(qwk_step_f64, 8, 64, true, qw::kEncReal)
QW_STEP_KERNEL(qwk_step_c1, 1, 0, false, qw::kEncComplex)
QW_STEP_KERNEL(qwk_step_c2, 2, 0, false, qw::kEncComplex)
QW_STEP_KERNEL(qwk_step_c4, 4, 0, false, qw::kEncComplex)
QW_STEP_KERNEL(qwk_step_c8, 8, 0, false, qw::kEncComplex)
QW_STEP_KERNEL(qwk_step_x1, 1, 0, false, qw::kEncAngle)
QW_STEP_KERNEL(qwk_step_x2, 2, 0, false, qw::kEncAngle)
QW_STEP_KERNEL(qwk_step_x4, 4, 0, false, qw::kEncAngle)
QW_STEP_KERNEL(qwk_step_x8, 8, 0, false, qw::kEncAngle)
QW_STEP_KERNEL(qwk_step_h1, 1, 0, true, qw::kEncComplex)
QW_STEP_KERNEL(qwk_step_h2, 2, 0, true, qw::kEncComplex)
QW_STEP_KERNEL(qwk_step_h4, 4, 0, true, qw::kEncComplex)
QW_STEP_KERNEL(qwk_step_h8, 8, 0, true, qw::kEncComplex)
QW_STEP_KERNEL(qwk_step_y1, 1, 0, true, qw::kEncAngle)
QW_STEP_KERNEL(qwk_step_y2, 2, 0, true, qw::kEncAngle)
QW_STEP_KERNEL(qwk_step_y4, 4, 0, true, qw::kEncAngle)
QW_STEP_KERNEL(qwk_step_y8, 8, 0, true, qw::kEncAngle)
QW_STEP_KERNEL(qwk_step_k1, 1, 1, true, qw::kEncComplex)
QW_STEP_KERNEL(qwk_step_k2, 1, 2, true, qw::kEncComplex)
QW_STEP_KERNEL(qwk_step_k4, 1, 4, true, qw::kEncComplex)
QW_STEP_KERNEL(qwk_step_k8, 1, 8, true, qw::kEncComplex)
QW_STEP_KERNEL(qwk_step_k16, 2, 16, true, qw::kEncComplex)
QW_STEP_KERNEL(qwk_step_k32, 4, 32, true, qw::kEncComplex)
QW_STEP_KERNEL(qwk_step_k64, 8, 64, true, qw::kEncComplex)
QW_STEP_KERNEL_W(qwk_step_f16w, 1, 16, qw::kEncReal)
QW_STEP_KERNEL_W(qwk_step_f32w, 2, 32, qw::kEncReal)
QW_STEP_KERNEL_W(qwk_step_f64w, 4, 64, qw::kEncReal)
QW_STEP_KERNEL_W(qwk_step_k16w, 1, 16, qw::kEncComplex)
QW_STEP_KERNEL_W(qwk_step_k32w, 2, 32, qw::kEncComplex)
QW_STEP_KERNEL_W(qwk_step_k64w, 4, 64, qw::kEncComplex)
#undef QW_STEP_KERNEL
#undef QW_STEP_KERNEL_W

namespace qw {

// ----------------------------------------------------------------- real amplitudes
// A real matrix whose negative values pair with negative values (a slot of
// value a < 0 has a partner, of value < 0: true of symmetric matrices) and a
// real b: every amplitude is then real or imaginary by its cell.  f = +-i
// sqrt|a| for a < 0 and real otherwise, and g is real.  By induction over the
// steps, the R0 cell of a slot of negative value holds i r and every other
// cell a real r.  T~ puts b f / sqrt(s) into R0; the group sum
// c = sum conj(f) x0 + g x1 is real, since conj(+-i q) (i r) = +-q r; the
// reflected R0 output (2/s) c f - x0 lands in the partner's R0, whose value
// is negative too; the rest is real.  So each cell keeps one double: r.  With
// f' = +-q (the sign of the +-i rule) for a < 0 and f' = f otherwise, the
// step reads c = sum f' r0 + g r1 and writes (2/s) c f' - r0 and
// (2/s) c g - r1: the complex step with the i's taken out.  The planes then
// hold doubles, 8 bytes per cell instead of 16; StepArgs::real is set and the
// plane pointers of StepArgs::in/out point at double arrays of the same
// layout.  These kernels have the f kernels' conditions (one s for every
// instance) or the g kernels' (mixed s): one pass, every row exists, the
// walk step only, and an empty list (T~ starts).

__device__ __forceinline__ double prune_r(double v, double tau, unsigned& cnt) {
  if (fabs(v) > tau) {
    ++cnt;
    return v;
  }
  return 0.0;
}

// Rows split over K wavefronts (the real step kernels of one s >= kSplitMinS,
// in workgroups of a multiple of K wavefronts; K = 2 with eight lanes per
// row, K = 4 with sixteen).  With eight lanes per row a wavefront covers 8 rows
// (four with sixteen), so each of its loads and stores touches 64-byte
// (32-byte) runs of the slot-position-major planes, part of a 128-byte line.
// Here wavefronts Kp .. Kp + K - 1 of an instance share rows 16p .. 16p + 15:
// wavefront Kp + q takes slot positions q s/K .. (q + 1) s/K - 1, lane
// g * 16 + jj holds positions q s/K + g sl + i (i < sl, the same slots per
// lane as the whole-row mapping) of row 16p + jj, so every access covers
// 128-byte runs with as many wavefronts as before (the paper's shape E,
// 16384 rows with s = 64: 9.35 -> 8.92 us per step with eight lanes per row,
// 8.3 us with sixteen, which whole rows had made the slower tile at 11.7 us).  The row sum: the four
// lanes of a row in the wavefront (lane ^ 16, lane ^ 32), then the K parts
// through LDS, added in one order by every wavefront of the group.  A group
// lies in one workgroup (wavefronts per workgroup a multiple of K, instances
// of N K / 16 wavefronts each, N >= s >= 16) and is either inside the slots
// or past them as a whole, so all of its wavefronts reach the barrier or
// none does.
// The smallest s with the split mapping.  For s = 16 and 32 the same split
// left shape D unchanged (3.23-3.25 us per step) and made shape C's
// 64-thread whole-row launches 5 % slower (2.11 -> 2.22 us, A/B on one box:
// the kernel holding both mappings), so those kernels keep whole rows only.
constexpr int kSplitMinS = 64;
template <int S, int K>
__device__ __forceinline__ Lanes lanes_split(const Matrix& m, int64_t w, int lane) {
  Lanes x;
  x.inst = m.ninst == 1 ? 0 : uload(m.wave_inst + w);
  x.I = inst_uniform(m, x.inst);
  const int64_t lw = w - x.I.wave_base;
  x.rpw_log = 4;  // 16 rows of the wavefront in the low lane bits
  x.h = int((lw % K) << 2) + (lane >> 4);
  x.j = int(((lw / K) << 4) + (lane & 15));
  x.live = true;
  return x;
}
template <int K>
__device__ __forceinline__ double join_parts(double c, int lane) {
  __shared__ double part[kMaxBlock / kWave][16];
  const int wib = int(threadIdx.x) >> 6;
  if (lane < 16) part[wib][lane] = c;
  __syncthreads();
  const int first = wib & ~(K - 1);
  double t = part[first][lane & 15];
#pragma unroll
  for (int q = 1; q < K; ++q) t += part[first + q][lane & 15];
  return t;
}

// S: s of every instance, or 0 (read per instance, slots per lane <= SLM;
// slots of value 0 are skipped as in step_wave when StepArgs::zskip is set).
// EQ0: when Q0 of a slot without a partner is read (see below); both forms
// are correct for every matrix, the launcher takes the faster one.
// The same join for two sums at once (the adjoint kernels' c and d).
template <int K>
__device__ __forceinline__ double2 join_parts2(double2 cd, int lane) {
  __shared__ double2 part2[kMaxBlock / kWave][16];
  const int wib = int(threadIdx.x) >> 6;
  if (lane < 16) part2[wib][lane] = cd;
  __syncthreads();
  const int first = wib & ~(K - 1);
  double2 t = part2[first][lane & 15];
#pragma unroll
  for (int q = 1; q < K; ++q) {
    const double2 u = part2[first + q][lane & 15];
    t = make_double2(t.x + u.x, t.y + u.y);
  }
  return t;
}

// K > 1: rows split over K wavefronts (lanes_split; S >= kSplitMinS, K = 2
// for W = 0, 4 for W = 1).
template <bool ACC, int SLM, int S, int ENC, int W = 0, bool EQ0 = false, int K = 1>
__device__ __forceinline__ unsigned step_wave_real(const StepArgs& a, int64_t w, int lane, double coef) {
  static_assert(K == 1 || (S >= 16 && K == (W ? 4 : 2) && S / (4 * K) == Shape<S, W>::sl),
                "the split mapping keeps the slots per lane of the whole-row mapping");
  const Lanes x = K > 1 ? lanes_split<S, K>(a.m, w, lane) : lanes_of<S, true, W>(a.m, w, lane);
  const int sl = S ? Shape<S, W>::sl : (SLM == 1 ? 1 : x.I.sl);
  const int64_t base = x.I.item_base;
  const double* R0 = reinterpret_cast<const double*>(a.in.R0);
  const double* R1 = reinterpret_cast<const double*>(a.in.R1);
  const double* Q0 = reinterpret_cast<const double*>(a.in.Q0);
  double* oR0 = reinterpret_cast<double*>(a.out.R0);
  double* oQ0 = reinterpret_cast<double*>(a.out.Q0);
  double* oQ1 = reinterpret_cast<double*>(a.out.Q1);
  int64_t h[SLM];
  StepSlot rc[SLM];
  double x0[SLM], x1[SLM], f[SLM], g[SLM], y0[SLM];
  bool zero[SLM];
  // Kernels of one s with at most two slots per lane read f' and g from the
  // rotation table (Matrix::sfg, 16 bytes per slot) instead of the value
  // (8 bytes) and two square roots: the cache-resident steps are bound by
  // their chain of dependent operations (per step, each pair of builds timed
  // back to back on one GPU:
  // G(16384, 8) 2.58 -> 2.45 us, C -6 %, D with sixteen lanes -4 %).  With
  // more slots per lane, or mixed s, the step is bound by bandwidth and the
  // extra bytes cost more (shape E +7 %, the 256-instance batch +9 %).
  constexpr bool kTab = S != 0 && SLM <= 2;
  double2 fgv[SLM];
  // Q0 of a slot without a partner (fillers at the edge of a band).  EQ0:
  // issued with the other loads, not after the group sum, where a second
  // round trip at the end of the wavefront cost 0.9 us per step on the
  // paper's shape E.  Matrices where every slot has a partner (no Q0 cells)
  // take the other form: the early load's code alone cost 6 % at 16384 x 8.
  const bool skip0 = S == 0 && a.zskip;
  if constexpr (S != 0) {
    // One s for every instance: the loads come in two rounds.  First those
    // of every slot that depend on nothing loaded (the record, R1, R0), all
    // issued before any is used; then the Q0 loads, which depend on a record
    // just read.  In one loop the compiler waited for each slot's record
    // before issuing the next slot's loads: a memory round trip per slot
    // held by the lane instead of two in all (shape E: 9.9 -> 9.4 us per
    // step; B 2.27 -> 2.20, D 3.97 -> 3.87).  The first round keeps the words
    // as loaded; they are decoded and scaled in the second.
    uint32_t link[SLM];
#pragma unroll
    for (int i = 0; i < SLM; ++i) {
      if (i < sl) {
        h[i] = base + (int64_t(x.h * sl + i) << x.I.nlog) + x.j;
        link[i] = a.m.slink[h[i]];
        if constexpr (kTab) {
          fgv[i] = reinterpret_cast<const double2*>(a.m.sfg)[h[i]];
          rc[i].val = 0.0;  // not read: the table holds the rotation
        } else {
          rc[i].val = a.m.sval[h[i]];
        }
        x1[i] = R1[h[i]];
        x0[i] = R0[h[i]];
      }
    }
    asm volatile("" ::: "memory");  // the second round's loads stay behind all of the first's
#pragma unroll
    for (int i = 0; i < SLM; ++i) {
      if (i < sl) {
        rc[i].part = int(link[i] & 0x7fffffffu) - 1;  // as step_rec
        rc[i].upper = (link[i] >> 31) == 0u;
        x1[i] *= a.in.r1s;
        zero[i] = false;
        y0[i] = 0.0;
        if (EQ0 && rc[i].part < 0) y0[i] = Q0[h[i]];
      }
    }
  } else {
    // Mixed s (the batch): one loop, slot after slot.  The two rounds above
    // made the HBM-bound 256-instance batch 0.5-1.7 % slower (26.6 against
    // 26.1-26.4 us per step, both builds timed back to back on one GPU).
#pragma unroll
    for (int i = 0; i < SLM; ++i) {
      if (i < sl) {
        h[i] = base + (int64_t(x.h * sl + i) << x.I.nlog) + x.j;
        rc[i] = step_rec(a.m, h[i]);
        x1[i] = R1[h[i]] * a.in.r1s;
        zero[i] = skip0 && rc[i].val == 0.0;
        x0[i] = zero[i] ? 0.0 : R0[h[i]];
        y0[i] = 0.0;
        if (EQ0 && !zero[i] && rc[i].part < 0) y0[i] = Q0[h[i]];
      }
    }
  }
  // The solver's y_j, loaded with the data: it is not needed before the
  // group sum.
  double* yp = nullptr;
  double yv = 0.0;
  if (ACC && x.h == 0) {
    yp = reinterpret_cast<double*>(a.yacc + x.I.jbase + x.j);
    yv = *yp;
  }
  double c = 0.0;
#pragma unroll
  for (int i = 0; i < SLM; ++i) {
    if (i < sl) {
      if constexpr (kTab) {
        f[i] = fgv[i].x;
        g[i] = fgv[i].y;
      } else {
        double q;
        if (ENC == kEncAngle) {
          sincospi(fabs(rc[i].val), &q, &g[i]);
        } else {
          q = sqrt(fabs(rc[i].val));
          g[i] = sqrt(1.0 - fabs(rc[i].val));
        }
        f[i] = rc[i].val < 0.0 && !rc[i].upper ? -q : q;  // f' (the +-i rule's sign for a < 0)
      }
      c += f[i] * x0[i] + x1[i] * g[i];
    }
  }
  c = row_sum_r<SLM>(c, x.rpw_log);
  if constexpr (K > 1) c = join_parts<K>(c, lane);
  if (ACC && x.h == 0) *yp = yv + coef * (c * x.I.inv_sqrt_s);  // the group sum is real: only Re y_j moves
  const double tc = c * two_over_s<S>(x.I);
  unsigned cnt = 0;
#pragma unroll
  for (int i = 0; i < SLM; ++i) {
    if (i < sl) {
      const double o0 = tc * f[i] - x0[i];
      const double o1 = tc * g[i] - x1[i];
      unsigned q1 = 0;
      oQ1[h[i]] = prune_r(o1, a.tau, q1);
      cnt += 2 * q1;  // counted as in write_slot
      if (zero[i]) continue;
      if (rc[i].part >= 0) {
        oR0[base + rc[i].part] = prune_r(o0, a.tau, cnt);
      } else {
        oQ0[h[i]] = prune_r(o0, a.tau, cnt);
        oR0[h[i]] = prune_r(EQ0 ? -y0[i] : -Q0[h[i]], a.tau, cnt);
      }
    }
  }
  return cnt;
}

// One wavefront's step and its branch count.
template <bool ACC, int SLM, int S, int ENC, int W, bool EQ0, int K>
__device__ __forceinline__ void step_counted(const StepArgs& a, int64_t w, int lane, int64_t wpb) {
  const double coef = ACC ? *a.coef : 0.0;
  const int64_t cidx = wave_counter(wpb);
  if (a.acc == nullptr) {  // the solver's private walk keeps no counts
    (void)step_wave_real<ACC, SLM, S, ENC, W, EQ0, K>(a, w, lane, coef);
    return;
  }
  const unsigned long long prev = a.acc[cidx];
  const unsigned long long v =
      wave_sum_bits<CountBits<SLM>::value>(step_wave_real<ACC, SLM, S, ENC, W, EQ0, K>(a, w, lane, coef));
  if (lane == 0) a.acc[cidx] = prev + v;
}

// XB: the row blocks numbered by XCD (xcd_row_block; the _x kernels, which
// the launcher takes when Matrix::xcd > 0).  A run-time choice in one kernel
// cost the plain numbering 1-3 % per step (its arguments and arithmetic
// reordered the loads of the prologue), so each numbering has kernels of its
// own.
template <bool ACC, int SLM, int S, int ENC, int W = 0, bool EQ0 = false, bool XB = false>
__device__ __forceinline__ void step_body_real(const StepArgs& a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wpb = XB ? int64_t(a.wpb & 0xff) : int64_t(a.wpb);
  const int64_t blk = XB ? xcd_row_block(blockIdx.x, int64_t(a.wpb >> 8)) : int64_t(blockIdx.x);
  const int64_t w = uniform(int(blk * wpb + (threadIdx.x >> 6)));
  // The arguments the wavefront needs, in registers before the branch below:
  // otherwise they are loaded after it, one more scalar-load round trip
  // ahead of the data loads (2.67 against 2.60 us per step at 16384 x 8).
  asm volatile("" ::"s"(a.m.inst0.item_base), "s"(a.m.inst0.nlog), "s"(a.m.slink), "s"(a.m.sval), "s"(a.in.R0),
               "s"(a.in.R1), "s"(a.out.R0), "s"(a.out.Q1), "s"(a.in.r1s), "s"(a.tau), "s"(a.acc));
  asm volatile("" ::"s"(a.m.ninst), "s"(a.m.inst0.wave_base), "s"(a.m.inst0.s), "s"(a.m.inst0.N), "s"(a.in.Q0),
               "s"(a.out.Q0), "s"(a.m.inst0.inv_sqrt_s), "s"(a.m.inst0.jbase), "s"(a.m.inst), "s"(a.m.wave_inst));
  if (w >= a.m.waves) return;  // no list: nothing to do past the slots
  if constexpr (S >= kSplitMinS) {
    constexpr int K = W ? 4 : 2;
    if (wpb % K == 0) {  // groups of K wavefronts in each workgroup: rows split over the group
      step_counted<ACC, SLM, S, ENC, W, EQ0, K>(a, w, lane, wpb);
      return;
    }
  }
  step_counted<ACC, SLM, S, ENC, W, EQ0, 1>(a, w, lane, wpb);
}

// Plane conversions for the switch between the two representations.  With
// `val` (an R0 plane: the step kernels' values by home) the cells of slots of
// negative value are the imaginary ones; without, every cell is real.
extern "C" __global__ void __launch_bounds__(256) qwk_to_real(const double2* __restrict__ src, double* dst,
                                                              const double* __restrict__ val, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = val && val[i] < 0.0 ? src[i].y : src[i].x;
}
extern "C" __global__ void __launch_bounds__(256) qwk_to_complex(const double* __restrict__ src, double2* dst,
                                                                 const double* __restrict__ val, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = val && val[i] < 0.0 ? make_double2(0.0, src[i]) : make_double2(src[i], 0.0);
}

}  // namespace qw

// qwk_step_rS: one double per cell, FP64 values, s = S for every instance;
// qwk_step_tS: the same for fixed-point data; qwk_step_rgN / qwk_step_tgN:
// mixed s, up to N slots per lane (the g kernels' shapes).  The _acc twins
// fuse the solver's projection, as the other families' do; the _q forms read
// Q0 of unpartnered slots early (step_wave_real's EQ0).
#define QW_REAL_KERNEL_(NAME, ACC, SLM, S, ENC, W, EQ0, XB)                                          \
  extern "C" __global__ void __launch_bounds__(256) NAME(qw::StepArgs a) {                         \
    qw::step_body_real<ACC, SLM, S, ENC, W, EQ0, XB>(a);                                            \
  }
#define QW_REAL_KERNEL4_(NAME, SLM, S, ENC, W)                     \
  QW_REAL_KERNEL_(NAME, false, SLM, S, ENC, W, false, false)       \
  QW_REAL_KERNEL_(NAME##_acc, true, SLM, S, ENC, W, false, false)  \
  QW_REAL_KERNEL_(NAME##_q, false, SLM, S, ENC, W, true, false)    \
  QW_REAL_KERNEL_(NAME##_q_acc, true, SLM, S, ENC, W, true, false) \
  QW_REAL_KERNEL_(NAME##_x, false, SLM, S, ENC, W, false, true)    \
  QW_REAL_KERNEL_(NAME##_x_acc, true, SLM, S, ENC, W, false, true) \
  QW_REAL_KERNEL_(NAME##_x_q, false, SLM, S, ENC, W, true, true)   \
  QW_REAL_KERNEL_(NAME##_x_q_acc, true, SLM, S, ENC, W, true, true)
#define QW_REAL_KERNEL(NAME, SLM, S, ENC) QW_REAL_KERNEL4_(NAME, SLM, S, ENC, 0)
#define QW_REAL_KERNEL_W(NAME, SLM, S, ENC) QW_REAL_KERNEL4_(NAME, SLM, S, ENC, 1)
QW_REAL_KERNEL(qwk_step_r1, 1, 1, qw::kEncReal)
QW_REAL_KERNEL(qwk_step_r2, 1, 2, qw::kEncReal)
QW_REAL_KERNEL(qwk_step_r4, 1, 4, qw::kEncReal)
QW_REAL_KERNEL(qwk_step_r8, 1, 8, qw::kEncReal)
QW_REAL_KERNEL(qwk_step_r16, 2, 16, qw::kEncReal)
QW_REAL_KERNEL(qwk_step_r32, 4, 32, qw::kEncReal)
QW_REAL_KERNEL(qwk_step_r64, 8, 64, qw::kEncReal)
QW_REAL_KERNEL(qwk_step_t1, 1, 1, qw::kEncAngle)
QW_REAL_KERNEL(qwk_step_t2, 1, 2, qw::kEncAngle)
QW_REAL_KERNEL(qwk_step_t4, 1, 4, qw::kEncAngle)
QW_REAL_KERNEL(qwk_step_t8, 1, 8, qw::kEncAngle)
QW_REAL_KERNEL(qwk_step_t16, 2, 16, qw::kEncAngle)
QW_REAL_KERNEL(qwk_step_t32, 4, 32, qw::kEncAngle)
QW_REAL_KERNEL(qwk_step_t64, 8, 64, qw::kEncAngle)
QW_REAL_KERNEL(qwk_step_rg1, 1, 0, qw::kEncReal)
QW_REAL_KERNEL(qwk_step_rg2, 2, 0, qw::kEncReal)
QW_REAL_KERNEL(qwk_step_rg4, 4, 0, qw::kEncReal)
QW_REAL_KERNEL(qwk_step_rg8, 8, 0, qw::kEncReal)
QW_REAL_KERNEL(qwk_step_tg1, 1, 0, qw::kEncAngle)
QW_REAL_KERNEL(qwk_step_tg2, 2, 0, qw::kEncAngle)
QW_REAL_KERNEL(qwk_step_tg4, 4, 0, qw::kEncAngle)
QW_REAL_KERNEL(qwk_step_tg8, 8, 0, qw::kEncAngle)
QW_REAL_KERNEL_W(qwk_step_r16w, 1, 16, qw::kEncReal)
QW_REAL_KERNEL_W(qwk_step_r32w, 2, 32, qw::kEncReal)
QW_REAL_KERNEL_W(qwk_step_r64w, 4, 64, qw::kEncReal)
QW_REAL_KERNEL_W(qwk_step_t16w, 1, 16, qw::kEncAngle)
QW_REAL_KERNEL_W(qwk_step_t32w, 2, 32, qw::kEncAngle)
QW_REAL_KERNEL_W(qwk_step_t64w, 4, 64, qw::kEncAngle)
#undef QW_REAL_KERNEL
#undef QW_REAL_KERNEL_W
#undef QW_REAL_KERNEL4_
#undef QW_REAL_KERNEL_


namespace qw {

// ----------------------------------------------------------------- QBS table
// rev = i_{col[q]}(j): where row j's slot q points back into its column's
// row (-1: filler or asymmetric pattern).  The record of slot (j, l) at its
// home holds col, the partner's home relative to the instance base
// (rev * N + col, or -1) and the value; the step kernels' record holds the
// partner, whether j <= col, and the value.

extern "C" __global__ void __launch_bounds__(256) qwk_qbs_table(Matrix m, SlotRec* rec, uint32_t* slink,
                                                                double* sval) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < m.items; it += stride) {
    const Inst I = m.inst[find_inst<&Inst::item_base>(m, it)];
    const int64_t local = it - I.item_base;
    if (local >= (int64_t(I.N) << I.hbits)) continue;
    const int j = int(local >> I.hbits);
    const int l = int(local & (I.s - 1));
    const int c = m.col[it];
    int p;
    SlotRec sr;
    sr.col = c;
    sr.part = qbs(m.col + I.item_base + (int64_t(c) << I.hbits), I.s, j, p) ? (p << I.nlog) + c : -1;
    sr.val = m.val[it];
    const int64_t hh = home(I, j, l);
    rec[hh] = sr;
    slink[hh] = uint32_t(sr.part + 1) | (j > c ? 0x80000000u : 0u);  // part + 1 <= N s < 2^31
    sval[hh] = sr.val;
  }
}

// Matrix::sfg: the rotation of every slot (by home, padding included),
// computed from slink, sval and vim exactly as the step kernels compute it
// (step_wave_real; rot_cplx in step_wave), so a kernel that reads the table
// takes the same values bit for bit.
extern "C" __global__ void __launch_bounds__(256) qwk_rot_table(Matrix m, double* sfg) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t h = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; h < m.items; h += stride) {
    const StepSlot rc = step_rec(m, h);
    if (m.vim) {
      const Rot r = rot_cplx(rc.val, m.vim[h], rc.upper);
      sfg[4 * h] = r.f.x;
      sfg[4 * h + 1] = r.f.y;
      sfg[4 * h + 2] = r.g;
      sfg[4 * h + 3] = 0.0;
      continue;
    }
    double q, g;
    if (m.angles) {
      sincospi(fabs(rc.val), &q, &g);
    } else {
      q = sqrt(fabs(rc.val));
      g = sqrt(1.0 - fabs(rc.val));
    }
    sfg[2 * h] = rc.val < 0.0 && !rc.upper ? -q : q;
    sfg[2 * h + 1] = g;
  }
}

// ----------------------------------------------------------------- adjoint sweep step
// One reverse step of the gradient: the recomputed state Psi_t and the
// adjoint state Lambda_t (both kept S-conjugated, so that W^dagger acts as W)
// advance by one walk step, and every slot (j, l) accumulates
//   dL/dv_{jl} += 2 Re[ (2/s) ( c (conj(mu_0) f' + conj(mu_1) g')
//                              + conj(d) (conj(f') psi'_0 + g' psi'_1) ) ]
// with chi, mu the group amplitudes of Psi_t and Lambda_t, c, d their group
// sums, and psi' = (2/s) c phi - chi the forward state before the reflection
// of step t.  dv is indexed by home.

template <int SLM>
__device__ __forceinline__ void adjoint_wave(const AdjArgs& a, int64_t w, int lane, unsigned& cnt,
                                             unsigned& lcnt) {
  const Lanes x = lanes_of<0, false>(a.m, w, lane);
  const int sl = SLM == 1 ? 1 : x.I.sl;
  const int64_t base = x.I.item_base;
  int64_t h[SLM];
  SlotRec rc[SLM];
  double2 x0[SLM], x1[SLM], m0[SLM], m1[SLM];
  Rot r[SLM];
#pragma unroll
  for (int i = 0; i < SLM; ++i) {
    if (i < sl) {
      h[i] = base + (int64_t(x.h * sl + i) << x.I.nlog) + x.j;
      rc[i] = a.m.rec[h[i]];
      x0[i] = a.in.R0[h[i]];
      x1[i] = r1_of(a.in, h[i]);
      m0[i] = a.lin.R0[h[i]];
      m1[i] = r1_of(a.lin, h[i]);
    }
  }
  // complex values: the imaginary parts by home (one uniform test per
  // wavefront); the derivatives come with the rotation
  const double* vim = a.m.vim;
  Rot dra[SLM], drb[SLM];
  double2 c = zero2(), d = zero2();
#pragma unroll
  for (int i = 0; i < SLM; ++i) {
    if (i < sl) {
      if (vim)
        rot_and_derivs(rc[i].val, vim[h[i]], x.j, rc[i].col, r[i], dra[i], drb[i]);
      else
        r[i] = rotation(rc[i].val, x.j, rc[i].col);
      c = cadd(c, along(r[i], x0[i], x1[i]));
      d = cadd(d, along(r[i], m0[i], m1[i]));
    }
  }
  c = row_sum<SLM>(c, x.rpw_log);
  d = row_sum<SLM>(d, x.rpw_log);
  if (!x.live) return;
  const double t = two_over_s<0>(x.I);
  const double2 tc = cscale(c, t), td = cscale(d, t);
#pragma unroll
  for (int i = 0; i < SLM; ++i) {
    if (i < sl) {
      const double2 q0 = csub(cmul(tc, r[i].f), x0[i]);  // psi'
      const double2 q1 = csub(cscale(tc, r[i].g), x1[i]);
      const double2 w0 = csub(cmul(td, r[i].f), m0[i]);  // reflected adjoint
      const double2 w1 = csub(cscale(td, r[i].g), m1[i]);
      // c (conj(mu_0) f' + conj(mu_1) g') + conj(d) (conj(f') psi'_0 + g' psi'_1)
      // for the derivative (f', g') of the rotation by one real parameter
      const auto du = [&](const Rot& dr) {
        return cadd(cmul(c, cadd(cjmul(m0[i], dr.f), make_double2(m1[i].x * dr.g, -m1[i].y * dr.g))),
                    cjmul(d, cadd(cjmul(dr.f, q0), cscale(q1, dr.g))));
      };
      if (vim) {
        a.dv[h[i]] += 2.0 * t * du(dra[i]).x;
        a.dvi[h[i]] += 2.0 * t * du(drb[i]).x;
      } else {
        a.dv[h[i]] += 2.0 * t * du(rotation_deriv(rc[i].val, x.j, rc[i].col)).x;
      }
      write_slot(a.in, a.out, base, h[i], rc[i].part, q0, q1, true, a.tau, cnt);
      write_slot(a.lin, a.lout, base, h[i], rc[i].part, w0, w1, true, a.tau, lcnt);
    }
  }
}

template <int SLM>
__device__ __forceinline__ void adjoint_body(const AdjArgs& a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wpb = a.wpb;
  const int64_t lw = (int64_t(a.L.cnt) + kWave - 1) / kWave;
  const int64_t llw = (int64_t(a.LL.cnt) + kWave - 1) / kWave;
  const int64_t total = a.m.waves + lw + llw;
  const int64_t cidx = wave_counter(wpb);
  const unsigned long long prev = a.acc[cidx], lprev = a.lacc[cidx];
  unsigned cnt = 0, lcnt = 0;
  const int64_t wstride = int64_t(gridDim.x) * wpb;
  for (int64_t w = uniform(int(blockIdx.x * wpb + (threadIdx.x >> 6))); w < total; w += wstride) {
    if (w < a.m.waves)
      adjoint_wave<SLM>(a, w, lane, cnt, lcnt);
    else if (w < a.m.waves + lw)
      cnt += list_entry(a.L, (w - a.m.waves) * kWave + lane, a.m.nbits, true);
    else
      lcnt += list_entry(a.LL, (w - a.m.waves - lw) * kWave + lane, a.m.nbits, true);
  }
  const unsigned long long v = wave_sum(cnt), lv = wave_sum(lcnt);
  if (lane == 0) {
    a.acc[cidx] = prev + v;
    a.lacc[cidx] = lprev + lv;
  }
}

}  // namespace qw

extern "C" __global__ void __launch_bounds__(256) qwk_adjoint_s1(qw::AdjArgs a) { qw::adjoint_body<1>(a); }
extern "C" __global__ void __launch_bounds__(256) qwk_adjoint_s2(qw::AdjArgs a) { qw::adjoint_body<2>(a); }
extern "C" __global__ void __launch_bounds__(256) qwk_adjoint_s4(qw::AdjArgs a) { qw::adjoint_body<4>(a); }
extern "C" __global__ void __launch_bounds__(256) qwk_adjoint_s8(qw::AdjArgs a) { qw::adjoint_body<8>(a); }

namespace qw {

// ----------------------------------------------------------------- adjoint sweep step, one double per cell
// The reverse step of adjoint_wave for a state on the 8-byte planes (both the
// recomputed state and the adjoint state: S-conjugation and the weighting
// diag(w) keep every cell real or imaginary by the rule of step_wave_real).
// With f' = +-sqrt|a| (the sign of the +-i rule for a < 0) and
// f_d' = df'/d|a| taken the same way (f_d = i f_d' for a < 0), every term of
// the complex formula is real:
//   c = sum f' x0 + g x1,  d = sum f' m0 + g m1  (row sums over the group),
//   p = (2/s) c (f', g) - x  (the forward state's outputs of this step),
//   dL/dv += 2 (2/s) [ c (m0 f_d' + m1 g_d) + d (f_d' p0 + g_d p1) ],
// and the outputs are the real step's for both states.  One pass over the
// wavefronts (every row exists, empty lists).  Returns the recomputed
// state's kept outputs, counted as the step kernels count them.
// K > 1: rows split over K wavefronts, as in step_wave_real.
template <int SLM, int S, int W = 0, bool EQ0 = false, int K = 1>
__device__ __forceinline__ unsigned adjoint_wave_real(const AdjArgs& a, int64_t w, int lane) {
  static_assert(K == 1 || (S >= 16 && K == (W ? 4 : 2) && S / (4 * K) == Shape<S, W>::sl),
                "the split mapping keeps the slots per lane of the whole-row mapping");
  const Lanes x = K > 1 ? lanes_split<S, K>(a.m, w, lane) : lanes_of<S, true, W>(a.m, w, lane);
  const int sl = S ? Shape<S, W>::sl : (SLM == 1 ? 1 : x.I.sl);
  const int64_t base = x.I.item_base;
  const double* R0 = reinterpret_cast<const double*>(a.in.R0);
  const double* R1 = reinterpret_cast<const double*>(a.in.R1);
  const double* Q0 = reinterpret_cast<const double*>(a.in.Q0);
  const double* LR0 = reinterpret_cast<const double*>(a.lin.R0);
  const double* LR1 = reinterpret_cast<const double*>(a.lin.R1);
  const double* LQ0 = reinterpret_cast<const double*>(a.lin.Q0);
  int64_t h[SLM];
  StepSlot rc[SLM];
  double x0[SLM], x1[SLM], m0[SLM], m1[SLM], f[SLM], g[SLM], y0[SLM], z0[SLM];
  uint32_t link[SLM];
#pragma unroll
  for (int i = 0; i < SLM; ++i) {  // words as loaded, in two rounds (as in step_wave_real)
    if (i < sl) {
      h[i] = base + (int64_t(x.h * sl + i) << x.I.nlog) + x.j;
      link[i] = a.m.slink[h[i]];
      rc[i].val = a.m.sval[h[i]];
      x1[i] = R1[h[i]];
      x0[i] = R0[h[i]];
      m1[i] = LR1[h[i]];
      m0[i] = LR0[h[i]];
    }
  }
  asm volatile("" ::: "memory");
#pragma unroll
  for (int i = 0; i < SLM; ++i) {  // the loads that depend on a record, after all others
    if (i < sl) {
      rc[i].part = int(link[i] & 0x7fffffffu) - 1;  // as step_rec
      rc[i].upper = (link[i] >> 31) == 0u;
      x1[i] *= a.in.r1s;
      m1[i] *= a.lin.r1s;
      y0[i] = z0[i] = 0.0;  // Q0 of slots without a partner, early or late (step_wave_real's EQ0)
      if (EQ0 && rc[i].part < 0) {
        y0[i] = Q0[h[i]];
        z0[i] = LQ0[h[i]];
      }
    }
  }
  double c = 0.0, d = 0.0;
#pragma unroll
  for (int i = 0; i < SLM; ++i) {
    if (i < sl) {
      const double q = sqrt(fabs(rc[i].val));
      g[i] = sqrt(1.0 - fabs(rc[i].val));
      f[i] = rc[i].val < 0.0 && !rc[i].upper ? -q : q;
      c += f[i] * x0[i] + x1[i] * g[i];
      d += f[i] * m0[i] + m1[i] * g[i];
    }
  }
  c = row_sum_r<SLM>(c, x.rpw_log);
  d = row_sum_r<SLM>(d, x.rpw_log);
  if constexpr (K > 1) {
    const double2 cd = join_parts2<K>(make_double2(c, d), lane);
    c = cd.x;
    d = cd.y;
  }
  const double t = two_over_s<S>(x.I);
  const double tc = c * t, td = d * t;
  double* oR0 = reinterpret_cast<double*>(a.out.R0);
  double* oQ0 = reinterpret_cast<double*>(a.out.Q0);
  double* oQ1 = reinterpret_cast<double*>(a.out.Q1);
  double* lR0 = reinterpret_cast<double*>(a.lout.R0);
  double* lQ0 = reinterpret_cast<double*>(a.lout.Q0);
  double* lQ1 = reinterpret_cast<double*>(a.lout.Q1);
  unsigned cnt = 0, unused = 0;
#pragma unroll
  for (int i = 0; i < SLM; ++i) {
    if (i < sl) {
      const double v = rc[i].val;
      const double p0 = tc * f[i] - x0[i], p1 = tc * g[i] - x1[i];
      const double w0 = td * f[i] - m0[i], w1 = td * g[i] - m1[i];
      // df'/da and dg/da (not finite at a = 0 and |a| = 1)
      const double fq = 0.5 / sqrt(fabs(v));
      const double fd = v > 0.0 ? fq : (v < 0.0 ? (rc[i].upper ? -fq : fq) : __builtin_inf());
      const double gd = (v > 0.0 ? -0.5 : (v < 0.0 ? 0.5 : 0.0)) / sqrt(1.0 - fabs(v));
      const double u = c * (m0[i] * fd + m1[i] * gd) + d * (fd * p0 + gd * p1);
      a.dv[h[i]] += 2.0 * t * u;
      unsigned q1 = 0;
      oQ1[h[i]] = prune_r(p1, a.tau, q1);
      cnt += 2 * q1;  // counted as in write_slot
      lQ1[h[i]] = prune_r(w1, a.tau, unused);
      if (rc[i].part >= 0) {
        oR0[base + rc[i].part] = prune_r(p0, a.tau, cnt);
        lR0[base + rc[i].part] = prune_r(w0, a.tau, unused);
      } else {
        oQ0[h[i]] = prune_r(p0, a.tau, cnt);
        oR0[h[i]] = prune_r(EQ0 ? -y0[i] : -Q0[h[i]], a.tau, cnt);
        lQ0[h[i]] = prune_r(w0, a.tau, unused);
        lR0[h[i]] = prune_r(EQ0 ? -z0[i] : -LQ0[h[i]], a.tau, unused);
      }
    }
  }
  return cnt;
}

// XB: the row blocks numbered by XCD (the _x kernels; see step_body_real).
template <int SLM, int S, int W = 0, bool EQ0 = false, bool XB = false>
__device__ __forceinline__ void adjoint_body_real(const AdjArgs& a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wpb = XB ? int64_t(a.wpb & 0xff) : int64_t(a.wpb);
  const int64_t blk = XB ? xcd_row_block(blockIdx.x, int64_t(a.wpb >> 8)) : int64_t(blockIdx.x);
  const int64_t w = uniform(int(blk * wpb + (threadIdx.x >> 6)));
  if (w >= a.m.waves) return;
  const int64_t cidx = wave_counter(wpb);
  const unsigned long long prev = a.acc ? a.acc[cidx] : 0ull;
  unsigned cnt;
  if constexpr (S >= kSplitMinS) {
    constexpr int K = W ? 4 : 2;
    // groups of K wavefronts in each workgroup: rows split over the group
    cnt = wpb % K == 0 ? adjoint_wave_real<SLM, S, W, EQ0, K>(a, w, lane)
                       : adjoint_wave_real<SLM, S, W, EQ0, 1>(a, w, lane);
  } else {
    cnt = adjoint_wave_real<SLM, S, W, EQ0, 1>(a, w, lane);
  }
  if (a.acc) {
    const unsigned long long v = wave_sum_bits<CountBits<SLM>::value>(cnt);
    if (lane == 0) a.acc[cidx] = prev + v;
  }
}

}  // namespace qw

// qwk_adjoint_rS: s = S for every instance; qwk_adjoint_rgN: mixed s, up to N
// slots per lane; qwk_adjoint_rSw: 16 lanes per row (Matrix::wide).
#define QW_ADJ_REAL_KERNEL(NAME, SLM, S, W)                                                       \
  extern "C" __global__ void __launch_bounds__(256) NAME(qw::AdjArgs a) {                       \
    qw::adjoint_body_real<SLM, S, W, false>(a);                                                  \
  }                                                                                              \
  extern "C" __global__ void __launch_bounds__(256) NAME##_q(qw::AdjArgs a) { qw::adjoint_body_real<SLM, S, W, true>(a); } \
  extern "C" __global__ void __launch_bounds__(256) NAME##_x(qw::AdjArgs a) {                   \
    qw::adjoint_body_real<SLM, S, W, false, true>(a);                                            \
  }                                                                                              \
  extern "C" __global__ void __launch_bounds__(256) NAME##_x_q(qw::AdjArgs a) {                 \
    qw::adjoint_body_real<SLM, S, W, true, true>(a);                                             \
  }
QW_ADJ_REAL_KERNEL(qwk_adjoint_r1, 1, 1, 0)
QW_ADJ_REAL_KERNEL(qwk_adjoint_r2, 1, 2, 0)
QW_ADJ_REAL_KERNEL(qwk_adjoint_r4, 1, 4, 0)
QW_ADJ_REAL_KERNEL(qwk_adjoint_r8, 1, 8, 0)
QW_ADJ_REAL_KERNEL(qwk_adjoint_r16, 2, 16, 0)
QW_ADJ_REAL_KERNEL(qwk_adjoint_r32, 4, 32, 0)
QW_ADJ_REAL_KERNEL(qwk_adjoint_r64, 8, 64, 0)
QW_ADJ_REAL_KERNEL(qwk_adjoint_rg1, 1, 0, 0)
QW_ADJ_REAL_KERNEL(qwk_adjoint_rg2, 2, 0, 0)
QW_ADJ_REAL_KERNEL(qwk_adjoint_rg4, 4, 0, 0)
QW_ADJ_REAL_KERNEL(qwk_adjoint_rg8, 8, 0, 0)
QW_ADJ_REAL_KERNEL(qwk_adjoint_r16w, 1, 16, 1)
QW_ADJ_REAL_KERNEL(qwk_adjoint_r32w, 2, 32, 1)
QW_ADJ_REAL_KERNEL(qwk_adjoint_r64w, 4, 64, 1)
#undef QW_ADJ_REAL_KERNEL

namespace qw {

// ----------------------------------------------------------------- T~ |b~>
// T~ on |0, j, 0, 0, 0, 0> gives the group of j with amplitudes b_j phi_j:
// slot (j, l) receives b_j f/sqrt(s) and b_j g/sqrt(s) (Alg. 5).

extern "C" __global__ void __launch_bounds__(256) qwk_init(Matrix m, const double2* __restrict__ b, Slots out,
                                                           double tau) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < m.items; it += stride) {
    const Home x = home_item(m, it, it - (threadIdx.x & (kWave - 1)));
    if (!x.live) continue;
    const SlotRec rc = m.rec[it];
    const Rot r = rotation_of(m, rc.val, it, x.j, rc.col);
    const double2 bj = cscale(b[x.I.jbase + x.j], x.I.inv_sqrt_s);
    double2 o0 = cmul(r.f, bj);
    double2 o1 = cscale(bj, r.g);
    if (!kept(o0, tau)) o0 = zero2();
    if (!kept(o1, tau)) o1 = zero2();
    out.R0[it] = o0;
    out.R1[it] = cscale(o1, out.r1s);
  }
}

// ----------------------------------------------------------------- fill (zero)

extern "C" __global__ void qwk_fill(uint4* p, int64_t n16) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Partial sums of the per-wavefront counters: out[b] = the sum of
// a[i] over the grid-stride share of workgroup b (256 threads each).
extern "C" __global__ void __launch_bounds__(256) qwk_sum_counts(const unsigned long long* __restrict__ a, int64_t n,
                                                                  unsigned long long* out) {
  __shared__ unsigned long long part[256 / 64];
  unsigned long long v = 0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) v += a[i];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// The solver's coefficient window for a graph of `count` steps (one
// wavefront): window[i] = table[*base + i], then *base += count.  Every lane
// reads *base in the one load ahead of lane 0's store, so the update cannot
// overtake the reads.  With set >= 0 only *base = set.
extern "C" __global__ void __launch_bounds__(64) qwk_coef_window(const double* __restrict__ table, int64_t* base,
                                                                  double* window, int32_t count, int64_t set) {
  const int lane = threadIdx.x;
  if (set >= 0) {
    if (lane == 0) *base = set;
    return;
  }
  const int64_t b = *base;
  for (int i = lane; i < count; i += kWave) window[i] = table[b + i];
  if (lane == 0) *base = b + count;
}

// ----------------------------------------------------------------- measurements

// Over homes and the list: kind 0 = branch count, 1 = norm^2, 4 = branches
// of the Q1 plane, as per-block partials.
extern "C" __global__ void __launch_bounds__(256) qwk_measure(Matrix m, Slots st, List L, int32_t kind,
                                                              double* partial) {
  __shared__ double sh[16];
  const int64_t total = m.items + ((int64_t(L.cnt) + kWave - 1) & ~int64_t(kWave - 1));
  double acc = 0.0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < total; it += stride) {
    double2 v[4] = {zero2(), zero2(), zero2(), zero2()};
    if (it < m.items) {
      const Home x = home_item(m, it, it - (threadIdx.x & (kWave - 1)));
      if (x.live) {
        v[0] = st.R0[it];
        v[1] = r1_of(st, it);
        v[2] = st.Q0[it];
        v[3] = st.Q1[it];
      }
    } else if (it - m.items < int64_t(L.cnt)) {
      v[0] = L.amp[it - m.items];
    }
    if (kind == 4)
      acc += it < m.items ? double(nonzero(v[3])) : 0.0;
    else
      for (int i = 0; i < 4; ++i) acc += kind == 0 ? double(nonzero(v[i])) : norm2(v[i]);
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Over rows (one lane per row) and the list: kind 2 = j-register marginal
// (atomics into out, an N-vector that starts at zero), kind 3 = projection
// <psi~_j|state> (interleaved complex, stored).
extern "C" __global__ void __launch_bounds__(256) qwk_measure_rows(Matrix m, Slots st, List L, int32_t kind,
                                                                   double* out) {
  const int n = m.nbits;
  const uint64_t nm = (uint64_t(1) << n) - 1;
  const int64_t total = m.rows + int64_t(L.cnt);
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < total; it += stride) {
    if (it < m.rows) {
      const Row x = row_item(m, it);
      double p = 0.0;
      double2 c = zero2();
      for (int l = 0; l < x.I.s; ++l) {
        const int64_t h = home(x.I, x.j, l);
        const double2 p0 = st.R0[h], p1 = r1_of(st, h);
        if (kind == 2) {
          p += norm2(p0) + norm2(p1);
          const double sw = norm2(st.Q0[h]) + norm2(st.Q1[h]);
          if (sw != 0.0) atomicAdd(&out[x.I.jbase + m.rec[h].col], sw);
        } else {
          const SlotRec rc = m.rec[h];
          c = cadd(c, along(rotation_of(m, rc.val, h, x.j, rc.col), p0, p1));
        }
      }
      if (kind == 2) {
        if (p != 0.0) atomicAdd(&out[it], p);
      } else {
        out[2 * it] = c.x * x.I.inv_sqrt_s;
        out[2 * it + 1] = c.y * x.I.inv_sqrt_s;
      }
    } else if (kind == 2) {
      const int64_t e = it - m.rows;
      const double2 v = L.amp[e];
      const uint64_t key = L.key[e];
      const uint64_t inst = key >> (4 * n + 2);
      const int j = int((key >> (2 * n + 2)) & nm);
      if (inst < uint64_t(m.ninst) && norm2(v) != 0.0) atomicAdd(&out[m.inst[inst].jbase + j], norm2(v));
    }
  }
}

// ----------------------------------------------------------------- export / import

// Wave-level compacted append of up to four values per lane.
__device__ __forceinline__ void wave_append4(uint64_t* keys, double2* amps, uint32_t* count, uint32_t cap,
                                             const bool* app, const uint64_t* k, const double2* v) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  uint64_t mk[4];
  uint32_t nk[4], tot = 0;
  for (int i = 0; i < 4; ++i) {
    mk[i] = __ballot(app[i]);
    nk[i] = __popcll(mk[i]);
    tot += nk[i];
  }
  if (tot == 0) return;
  uint32_t base = 0;
  if (lane == 0) base = atomicAdd(count, tot);
  base = __shfl(base, 0);
  for (int i = 0; i < 4; ++i) {
    if (app[i]) {
      const uint32_t idx = base + __popcll(mk[i] & lt);
      if (idx < cap) {
        keys[idx] = k[i];
        amps[idx] = v[i];
      }
    }
    base += nk[i];
  }
}

extern "C" __global__ void __launch_bounds__(256) qwk_export(Matrix m, Slots st, List L, uint64_t* keys,
                                                             double2* amps, uint32_t* count, uint32_t cap) {
  const int n = m.nbits;
  const int64_t total = m.items + ((int64_t(L.cnt) + kWave - 1) & ~int64_t(kWave - 1));
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < total; it += stride) {
    bool app[4] = {false, false, false, false};
    uint64_t k[4] = {0, 0, 0, 0};
    double2 v[4] = {zero2(), zero2(), zero2(), zero2()};
    if (it < m.items) {
      const Home x = home_item(m, it, it - (threadIdx.x & (kWave - 1)));
      if (x.live) {
        const int colq = m.rec[it].col;
        v[0] = st.R0[it];
        v[1] = r1_of(st, it);
        v[2] = st.Q0[it];
        v[3] = st.Q1[it];
        for (int b2 = 0; b2 < 2; ++b2) {
          k[b2] = member_key(uint64_t(x.inst), n, x.j, colq, b2);
          k[2 + b2] = swapped_key(uint64_t(x.inst), n, x.j, colq, b2);
        }
        for (int i = 0; i < 4; ++i) app[i] = nonzero(v[i]);
      }
    } else {
      const int64_t e = it - m.items;
      if (e < int64_t(L.cnt)) {
        v[0] = L.amp[e];
        k[0] = L.key[e];
        app[0] = nonzero(v[0]);
      }
    }
    wave_append4(keys, amps, count, cap, app, k, v);
  }
}

// Static home of a key: 0..3 = plane R0, R1, Q0, Q1 (at home idx), 4 = none
// (the list).
__device__ __forceinline__ int home_of(const Matrix& m, uint64_t key, int64_t& idx) {
  const int n = m.nbits;
  const uint64_t nm = (uint64_t(1) << n) - 1;
  const int b2 = int(key & 1);
  const int k = int((key >> 1) & nm);
  const uint64_t kc = (key >> (n + 1)) & nm;
  const int b1 = int((key >> (2 * n + 1)) & 1);
  const int j = int((key >> (2 * n + 2)) & nm);
  const uint64_t jc = (key >> (3 * n + 2)) & nm;
  const uint64_t inst = key >> (4 * n + 2);
  if (jc != 0 || kc != 0 || inst >= uint64_t(m.ninst)) return 4;
  const Inst I = m.inst[inst];
  if (j >= I.N || k >= I.N) return 4;
  int p;
  if (b1 == 0 && qbs(m.col + I.item_base + (int64_t(j) << I.hbits), I.s, k, p)) {
    idx = home(I, j, p);
    return b2;
  }
  // (0, J, B1, 0, K, 0) = S K(q, B1) with q = (K, position of J in row K)
  if (b2 == 0 && qbs(m.col + I.item_base + (int64_t(k) << I.hbits), I.s, j, p)) {
    idx = home(I, k, p);
    return 2 + b1;
  }
  return 4;
}

extern "C" __global__ void __launch_bounds__(256) qwk_import(Matrix m, const uint64_t* keys, const double2* amps,
                                                             int64_t cnt, Slots out, List L, uint32_t* lcnt) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t total = (cnt + kWave - 1) & ~int64_t(kWave - 1);
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += stride) {
    bool app[4] = {false, false, false, false};
    uint64_t k[4] = {0, 0, 0, 0};
    double2 v[4] = {zero2(), zero2(), zero2(), zero2()};
    if (e < cnt) {
      k[0] = keys[e];
      v[0] = amps[e];
      int64_t idx = 0;
      const int h = home_of(m, k[0], idx);
      if (h == 0)
        out.R0[idx] = v[0];
      else if (h == 1)
        out.R1[idx] = cscale(v[0], out.r1s);
      else if (h == 2)
        out.Q0[idx] = v[0];
      else if (h == 3)
        out.Q1[idx] = v[0];
      else
        app[0] = true;
    }
    wave_append4(L.key, L.amp, lcnt, L.cap, app, k, v);
  }
}

// ----------------------------------------------------------------- export order
//
// The export hands branches over in key order; the compacted append leaves
// them in the order the wavefronts finished.  A least-significant-digit radix
// sort puts them in order on the GPU: 8-bit digits, one pass for each digit
// window that holds a bit on which some keys differ (bits every key shares
// cannot change the order, so those windows are skipped), each pass a stable
// counting sort over tiles of kSortTile keys: per-tile digit counts, their
// offsets, then a scatter that ranks equal digits in input order.

// bits[0] |= OR of the keys, bits[1] |= OR of their complements (so the
// bits on which the keys differ are bits[0] & bits[1]).  bits[] start at 0.
extern "C" __global__ void __launch_bounds__(256) qwk_key_bits(const uint64_t* keys, int64_t count,
                                                               unsigned long long* bits) {
  unsigned long long o = 0, z = 0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride) {
    o |= keys[i];
    z |= ~keys[i];
  }
  for (int d = 1; d < kWave; d <<= 1) {
    o |= __shfl_xor(o, d);
    z |= __shfl_xor(z, d);
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    atomicOr(&bits[0], o);
    atomicOr(&bits[1], z);
  }
}

// hist[tile * 256 + d] = keys of the tile whose digit (key >> shift) & 255 is d.
// One workgroup of 256 per tile.
extern "C" __global__ void __launch_bounds__(256) qwk_radix_hist(const uint64_t* keys, int64_t count, int shift,
                                                                 uint32_t* hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * kSortTile;
  for (int t = 0; t < kSortTile / 256; ++t) {
    const int64_t i = base + t * 256 + threadIdx.x;
    if (i < count) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[int64_t(blockIdx.x) * 256 + threadIdx.x] = h[threadIdx.x];
}

// One workgroup of 256 (thread d owns digit d): hist[tile * 256 + d] becomes
// the number of keys of digit d in the tiles before it, and digit_base[d] the
// number of keys of a smaller digit.
extern "C" __global__ void __launch_bounds__(256) qwk_radix_offsets(uint32_t* hist, int64_t tiles,
                                                                    uint32_t* digit_base) {
  __shared__ uint32_t s[256];
  const int d = threadIdx.x;
  uint32_t run = 0;
  for (int64_t b = 0; b < tiles; ++b) {
    const uint32_t c = hist[b * 256 + d];
    hist[b * 256 + d] = run;
    run += c;
  }
  s[d] = run;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {  // inclusive scan over the digits
    const uint32_t v = d >= off ? s[d - off] : 0u;
    __syncthreads();
    s[d] += v;
    __syncthreads();
  }
  digit_base[d] = s[d] - run;
}

// Scatter of one pass.  Keys are taken in input order: tile, then 256-key
// row t, then wavefront, then lane.  A lane's rank among the lanes of its
// wavefront with the same digit comes from eight ballots (one per digit
// bit); the counts of the wavefronts before it and of the rows before t
// (run[]) are kept in LDS.  Equal digits thus keep their input order, which
// makes each pass stable.
extern "C" __global__ void __launch_bounds__(256) qwk_radix_scatter(const uint64_t* kin, const double2* vin,
                                                                    int64_t count, int shift, const uint32_t* hist,
                                                                    const uint32_t* digit_base, uint64_t* kout,
                                                                    double2* vout) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wc[256 / kWave][256];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid >> 6;
  const uint64_t below = (uint64_t(1) << lane) - 1;
  run[tid] = hist[int64_t(blockIdx.x) * 256 + tid] + digit_base[tid];
  const int64_t base = int64_t(blockIdx.x) * kSortTile;
  for (int t = 0; t < kSortTile / 256; ++t) {
#pragma unroll
    for (int w = 0; w < 256 / kWave; ++w) wc[w][tid] = 0;
    __syncthreads();
    const int64_t i = base + t * 256 + tid;
    const bool ok = i < count;
    uint64_t k = 0;
    double2 v = zero2();
    int d = 0;
    if (ok) {
      k = kin[i];
      v = vin[i];
      d = int((k >> shift) & 255u);
    }
    uint64_t peer = __ballot(ok);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t set = __ballot((d >> bit) & 1);
      peer &= ((d >> bit) & 1) ? set : ~set;
    }
    const uint32_t rank = __popcll(peer & below);
    if (ok && rank == 0) wc[wave][d] = __popcll(peer);
    __syncthreads();
    if (ok) {
      uint32_t dst = run[d] + rank;
      for (int w = 0; w < wave; ++w) dst += wc[w][d];
      if (int64_t(dst) < count) {
        kout[dst] = k;
        vout[dst] = v;
      }
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < 256 / kWave; ++w) add += wc[w][tid];
    run[tid] += add;
  }
}

// re[i], im[i] = a[i] (the export's amplitudes into the caller's two arrays).
extern "C" __global__ void __launch_bounds__(256) qwk_split_amps(const double2* a, int64_t n, double* re, double* im) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double2 v = a[i];
    re[i] = v.x;
    im[i] = v.y;
  }
}

// ----------------------------------------------------------------- gradient set-up and finish

// Lambda = diag(w[k register]) Psi for a state kept S-conjugated (the j
// register of the true state is the k register of the stored one), and the
// loss sum_branches w |amp|^2 as per-block partials.  K(q, b2) has k = col[q];
// S K(q, b2) has k = j.
extern "C" __global__ void __launch_bounds__(256) qwk_weight(Matrix m, Slots in, List L, Slots out, List LL,
                                                             const double* w, double* partial) {
  __shared__ double sh[16];
  const int n = m.nbits;
  const uint64_t nm = (uint64_t(1) << n) - 1;
  const int64_t total = m.items + ((int64_t(L.cnt) + kWave - 1) & ~int64_t(kWave - 1));
  double acc = 0.0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < total; it += stride) {
    if (it < m.items) {
      const Home x = home_item(m, it, it - (threadIdx.x & (kWave - 1)));
      if (x.live) {
        const double wr = w[x.I.jbase + m.rec[it].col];
        const double wq = w[x.I.jbase + x.j];
        const double2 p0 = in.R0[it], p1 = r1_of(in, it), s0 = in.Q0[it], s1 = in.Q1[it];
        acc += wr * (norm2(p0) + norm2(p1)) + wq * (norm2(s0) + norm2(s1));
        out.R0[it] = cscale(p0, wr);
        out.R1[it] = cscale(p1, wr * out.r1s);
        out.Q0[it] = cscale(s0, wq);
        out.Q1[it] = cscale(s1, wq);
      }
    } else {
      const int64_t e = it - m.items;
      if (e < int64_t(L.cnt)) {
        const uint64_t key = L.key[e];
        const double2 p = L.amp[e];
        const uint64_t inst = key >> (4 * n + 2);
        const int k = int((key >> 1) & nm);
        const double wk = inst < uint64_t(m.ninst) ? w[m.inst[inst].jbase + k] : 0.0;
        acc += wk * norm2(p);
        LL.key[e] = key;
        LL.amp[e] = cscale(p, wk);
      }
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// ----------------------------------------------------------------- the same on one double per cell
// The swap S of a state on the 8-byte planes (a permutation of its cells:
// R0 to the partner's R0 or to its own Q0 and back, R1 to Q1, the R1 of the
// output being the input's Q1 plane with sign +1), one lane per home; the
// outputs are counted as the step kernels count them (acc may be NULL).
extern "C" __global__ void __launch_bounds__(256) qwk_swap_real(Matrix m, Slots in, Slots out,
                                                                unsigned long long* acc) {
  const double* R0 = reinterpret_cast<const double*>(in.R0);
  const double* R1 = reinterpret_cast<const double*>(in.R1);
  const double* Q0 = reinterpret_cast<const double*>(in.Q0);
  double* oR0 = reinterpret_cast<double*>(out.R0);
  double* oQ0 = reinterpret_cast<double*>(out.Q0);
  double* oQ1 = reinterpret_cast<double*>(out.Q1);
  const int64_t wpb = blockDim.x >> 6;
  const int64_t cidx = wave_counter(wpb);
  const unsigned long long prev = acc ? acc[cidx] : 0ull;
  unsigned cnt = 0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < m.items; it += stride) {
    const Home x = home_item(m, it, it - (threadIdx.x & (kWave - 1)));
    if (!x.live) continue;
    const double x0 = R0[it], x1 = R1[it] * in.r1s;
    const int part = int(m.slink[it] & 0x7fffffffu) - 1;
    oQ1[it] = x1;
    cnt += 2 * (x1 != 0.0);
    if (part >= 0) {
      oR0[x.I.item_base + part] = x0;
      cnt += x0 != 0.0;
    } else {
      const double y0 = Q0[it];
      oQ0[it] = x0;
      oR0[it] = y0;
      cnt += (x0 != 0.0) + (y0 != 0.0);
    }
  }
  const unsigned long long v = wave_sum(cnt);
  if (acc && (threadIdx.x & (kWave - 1)) == 0) acc[cidx] = prev + v;
}

// qwk_weight on the 8-byte planes: Lambda = diag(w[k register]) Psi and the
// loss as per-block partials.
extern "C" __global__ void __launch_bounds__(256) qwk_weight_real(Matrix m, Slots in, Slots out, const double* w,
                                                                  double* partial) {
  __shared__ double sh[16];
  const double* R0 = reinterpret_cast<const double*>(in.R0);
  const double* R1 = reinterpret_cast<const double*>(in.R1);
  const double* Q0 = reinterpret_cast<const double*>(in.Q0);
  const double* Q1 = reinterpret_cast<const double*>(in.Q1);
  double* oR0 = reinterpret_cast<double*>(out.R0);
  double* oR1 = reinterpret_cast<double*>(out.R1);
  double* oQ0 = reinterpret_cast<double*>(out.Q0);
  double* oQ1 = reinterpret_cast<double*>(out.Q1);
  double acc = 0.0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < m.items; it += stride) {
    const Home x = home_item(m, it, it - (threadIdx.x & (kWave - 1)));
    if (!x.live) continue;
    const double wr = w[x.I.jbase + m.rec[it].col];
    const double wq = w[x.I.jbase + x.j];
    const double p0 = R0[it], p1 = R1[it] * in.r1s, s0 = Q0[it], s1 = Q1[it];
    acc += wr * (p0 * p0 + p1 * p1) + wq * (s0 * s0 + s1 * s1);
    oR0[it] = p0 * wr;
    oR1[it] = p1 * (wr * out.r1s);
    oQ0[it] = s0 * wq;
    oQ1[it] = s1 * wq;
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Slots of a row that the seed kernels load together.
constexpr int kInitChunk = 8;

// qwk_grad_init on the 8-byte planes (a real b): with n the cells of lambda_0
// (imaginary R0 cells of slots of negative value held as their coefficient
// of i), dL/dv += 2 b_j (n0 f_d' + n1 g_d) / sqrt(s) and
// dL/db_j = 2 sum (f' n0 + g n1) / sqrt(s) (the real parts; the imaginary
// parts are 0).
extern "C" __global__ void __launch_bounds__(256) qwk_grad_init_real(Matrix m, Slots lam, const double2* b,
                                                                     double* dv, double2* db) {
  const double* N0 = reinterpret_cast<const double*>(lam.R0);
  const double* N1 = reinterpret_cast<const double*>(lam.R1);
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < m.rows; it += stride) {
    const Row x = row_item(m, it);
    const double bj = b[it].x;
    double c = 0.0;
    // eight slots at a time: every load of the chunk (dL/dv's old values
    // included) is issued before the first store, one round trip per chunk
    for (int l0 = 0; l0 < x.I.s; l0 += kInitChunk) {
      int64_t h[kInitChunk];
      double n0[kInitChunk], n1[kInitChunk], av[kInitChunk], dvo[kInitChunk];
      int col[kInitChunk];
#pragma unroll
      for (int i = 0; i < kInitChunk; ++i) {
        if (l0 + i < x.I.s) {
          h[i] = home(x.I, x.j, l0 + i);
          n0[i] = N0[h[i]];
          n1[i] = N1[h[i]] * lam.r1s;
          const SlotRec rc = m.rec[h[i]];
          av[i] = rc.val;
          col[i] = rc.col;
          dvo[i] = dv[h[i]];
        }
      }
#pragma unroll
      for (int i = 0; i < kInitChunk; ++i) {
        if (l0 + i < x.I.s) {
          const double a = av[i];
          const bool upper = x.j <= col[i];
          const double q = sqrt(fabs(a));
          const double f = a < 0.0 && !upper ? -q : q;
          const double g = sqrt(1.0 - fabs(a));
          const double fq = 0.5 / q;
          const double fd = a > 0.0 ? fq : (a < 0.0 ? (upper ? -fq : fq) : __builtin_inf());
          const double gd = (a > 0.0 ? -0.5 : (a < 0.0 ? 0.5 : 0.0)) / g;
          dv[h[i]] = dvo[i] + 2.0 * bj * (n0[i] * fd + n1[i] * gd) * x.I.inv_sqrt_s;
          c += f * n0[i] + g * n1[i];
        }
      }
    }
    db[it] = make_double2(2.0 * c * x.I.inv_sqrt_s, 0.0);
  }
}

// The gradient's results in the caller's order: gv[p] = dv[home[p]] for the
// CSC entries, br/bi[p] = db[row[p]] for the unpadded columns.
// With dvi (complex values): gvi[p] = dvi[home[p]] too.
extern "C" __global__ void __launch_bounds__(256) qwk_gather_grad(const double* __restrict__ dv,
                                                                  const int32_t* __restrict__ home, int64_t nnz,
                                                                  const double2* __restrict__ db,
                                                                  const int32_t* __restrict__ row, int64_t n,
                                                                  double* gv, double* br, double* bi,
                                                                  const double* __restrict__ dvi, double* gvi) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < nnz + n; p += stride) {
    if (p < nnz) {
      gv[p] = dv[home[p]];
      if (dvi) gvi[p] = dvi[home[p]];
    } else {
      const double2 v = db[row[p - nnz]];
      br[p - nnz] = v.x;
      bi[p - nnz] = v.y;
    }
  }
}

// Gradient through the initial T~ (one lane per row): psi_0 holds b_j phi_j
// in the group of j, so dL/dv_{jl} += 2 Re[b_j (conj(nu_0) f' + conj(nu_1) g')]
// / sqrt(s) with nu the group amplitudes of lambda_0, and
// dL/db_j = 2 <psi~_j|lambda_0>.  Complex values (Matrix::vim): the same
// with the derivatives by the real and the imaginary part, into dv and dvi.
extern "C" __global__ void __launch_bounds__(256) qwk_grad_init(Matrix m, Slots lam, const double2* b, double* dv,
                                                                double2* db, double* dvi) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < m.rows; it += stride) {
    const Row x = row_item(m, it);
    const double2 bj = b[it];
    double2 c = zero2();
    // eight slots at a time, every load of the chunk before the first store
    // (as in qwk_grad_init_real)
    for (int l0 = 0; l0 < x.I.s; l0 += kInitChunk) {
      int64_t h[kInitChunk];
      double2 n0[kInitChunk], n1[kInitChunk];
      double av[kInitChunk], vi[kInitChunk], dvo[kInitChunk], dvio[kInitChunk];
      int col[kInitChunk];
#pragma unroll
      for (int i = 0; i < kInitChunk; ++i) {
        if (l0 + i < x.I.s) {
          h[i] = home(x.I, x.j, l0 + i);
          n0[i] = lam.R0[h[i]];
          n1[i] = r1_of(lam, h[i]);
          const SlotRec rc = m.rec[h[i]];
          av[i] = rc.val;
          col[i] = rc.col;
          vi[i] = m.vim ? m.vim[h[i]] : 0.0;
          dvo[i] = dv[h[i]];
          dvio[i] = m.vim ? dvi[h[i]] : 0.0;
        }
      }
#pragma unroll
      for (int i = 0; i < kInitChunk; ++i) {
        if (l0 + i < x.I.s) {
          const auto du = [&](const Rot& d) {
            return cmul(bj, cadd(cjmul(n0[i], d.f), make_double2(n1[i].x * d.g, -n1[i].y * d.g)));
          };
          Rot r;
          if (m.vim) {
            Rot da, db2;
            rot_and_derivs(av[i], vi[i], x.j, col[i], r, da, db2);
            dv[h[i]] = dvo[i] + 2.0 * du(da).x * x.I.inv_sqrt_s;
            dvi[h[i]] = dvio[i] + 2.0 * du(db2).x * x.I.inv_sqrt_s;
          } else {
            r = rotation(av[i], x.j, col[i]);
            dv[h[i]] = dvo[i] + 2.0 * du(rotation_deriv(av[i], x.j, col[i])).x * x.I.inv_sqrt_s;
          }
          c = cadd(c, along(r, n0[i], n1[i]));
        }
      }
    }
    db[it] = cscale(c, 2.0 * x.I.inv_sqrt_s);
  }
}

}  // namespace qw
