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
// fixed address: R[q][b2] for K(q, b2), Q[q][b2] for a non-member S K(q, b2).
// One launch per step reads R_in and Q_in of its slot, reduces the group with
// wave shuffles, and writes each output to its address for the next step:
//   R_in  -> reflection -> Q_out[q][1] and R_out[q'][0] (or Q_out[q][0])
//   Q_in  -> negation   -> R_out[q][b2]
// Every output address receives exactly one write per step (0 when pruned),
// so there is no atomic, no compaction and no clearing pass; the result is
// independent of scheduling.  Branches outside that span (only from raw
// starts or imports) sit in a list that W maps in place to -S(key).
#include "qw_internal.h"

#include <hip/hip_runtime.h>

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
__device__ __forceinline__ Rot rotation(double a, int j, int k) {
  Rot r;
  const double q = sqrt(fabs(a));  // one square root, no divergent branch
  r.f = a >= 0.0 ? make_double2(q, 0.0) : make_double2(0.0, j <= k ? q : -q);
  r.g = sqrt(1.0 - fabs(a));
  return r;
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

template <int CTRL>
__device__ __forceinline__ double2 dpp_add(double2 v) {
  return make_double2(v.x + dpp<CTRL>(v.x), v.y + dpp<CTRL>(v.y));
}

// Sum over aligned groups of `width` lanes (width a power of two <= 64,
// uniform across the wavefront).  Each stage adds the value of a partner lane
// in the other half of the current block (DPP quad permutations and row
// mirrors inside rows of 16 lanes, lane shuffles beyond), so every lane of a
// group ends with the bitwise-identical sum.
__device__ __forceinline__ double2 group_sum(double2 v, int width) {
  if (width >= 2) v = dpp_add<0xB1>(v);   // quad_perm [1,0,3,2]: lane ^ 1
  if (width >= 4) v = dpp_add<0x4E>(v);   // quad_perm [2,3,0,1]: lane ^ 2
  if (width >= 8) v = dpp_add<0x141>(v);  // row_half_mirror: the other quad of 8
  if (width >= 16) v = dpp_add<0x140>(v); // row_mirror: the other 8 of 16
  for (int off = 16; off < width; off <<= 1) {
    v.x += __shfl_xor(v.x, off);
    v.y += __shfl_xor(v.y, off);
  }
  return v;
}

__device__ __forceinline__ int find_inst(const Matrix& m, int64_t item) {
  int lo = 0, hi = m.ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (m.inst[mid].item_base <= item)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
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

// Work item of a dense pass: instance (wave-uniform), slot, row, position.
struct Item {
  Inst I;
  int inst;
  int j, l;
  bool live;
};
// `first` is the first slot of the lane's wavefront (a wavefront never
// straddles two instances, so its instance is looked up once, uniformly).
__device__ __forceinline__ Item item_of(const Matrix& m, int64_t it, int64_t first) {
  Item x;
  x.inst = m.ninst == 1 ? 0 : __builtin_amdgcn_readfirstlane(find_inst(m, first));
  x.I = m.inst[x.inst];  // uniform address: scalar loads that overlap the data loads
  const int64_t local = it - x.I.item_base;
  x.live = local < int64_t(x.I.N) * x.I.s;
  x.l = int(local) & (x.I.s - 1);
  x.j = int(local >> x.I.hbits);
  return x;
}

__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v, unsigned long long* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  unsigned long long t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < int(blockDim.x >> 6); ++i) t += sh[i];
  return t;
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

// Outputs of one slot for the next step (shared by the step and adjoint
// kernels).  o0, o1: reflected group amplitudes of K(q, b2) before S;
// n0, n1: outputs of Q_in[q][b2] (already negated or not).
__device__ __forceinline__ void write_slot(const Slots& out, const Item& x, int64_t q, int colq, int pr, double2 o0,
                                           double2 o1, double2 n0, double2 n1) {
  out.Q[2 * q + 1] = o1;
  if (pr >= 0) {
    out.R[2 * (x.I.item_base + int64_t(colq) * x.I.s + pr)] = o0;
  } else {
    out.Q[2 * q] = o0;
    out.R[2 * q] = n0;
  }
  out.R[2 * q + 1] = n1;
}

// ----------------------------------------------------------------- walk step

// One lane per slot and b2 (groups of 2s lanes, s <= 32).  The data loads of
// a lane do not depend on each other or on the instance record: padding slots
// hold zeros (col 0, val 0, rev -1), so every load is in bounds and issued at
// once.  Returns the number of branches the lane wrote.
template <bool ACC>
__device__ __forceinline__ unsigned step_pairs(const Matrix& m, Slots in, Slots out, int32_t mode, double tau,
                                               double2* yacc, double coef, int64_t it, int64_t first) {
  const int64_t q = it >> 1;
  const int b2 = int(it & 1);
  const SlotRec rc = m.rec[q];
  const double2 x = in.R[it];
  const double2 y1 = in.Q[2 * q + 1];  // the b2 = 1 lane's input; same line as its partner lane's
  const Item xi = item_of(m, q, first);
  // the lane's component of sqrt(s) phi_j: f for b2 = 0, g for b2 = 1 (one square root)
  const double a = rc.val;
  const double sq = sqrt(b2 == 0 ? fabs(a) : 1.0 - fabs(a));
  const double2 w = (b2 == 1 || a >= 0.0) ? make_double2(sq, 0.0) : make_double2(0.0, xi.j <= rc.col ? sq : -sq);
  double2 y = b2 == 1 ? y1 : zero2();
  if (b2 == 0 && rc.rev < 0) y = in.Q[it];  // only slots whose swap is not a group member
  double2 o = x, n = y;
  if (mode == kStep) {
    const double2 c = group_sum(cjmul(w, x), 2 * xi.I.s);
    if (ACC && xi.live && xi.l == 0 && b2 == 0) {
      double2 yv = yacc[xi.I.jbase + xi.j];
      yv.x += coef * (c.x * xi.I.inv_sqrt_s);
      yv.y += coef * (c.y * xi.I.inv_sqrt_s);
      yacc[xi.I.jbase + xi.j] = yv;
    }
    o = csub(cmul(cscale(c, 2.0 / double(xi.I.s)), w), x);
    n = cneg(y);
  }
  unsigned cnt = 0;
  if (!xi.live) return 0;
  o = prune(o, tau, cnt);
  if (b2 == 1) {
    out.Q[it] = o;
    out.R[it] = prune(n, tau, cnt);
  } else if (rc.rev >= 0) {
    out.R[2 * (xi.I.item_base + int64_t(rc.col) * xi.I.s + rc.rev)] = o;
  } else {
    out.Q[it] = o;
    out.R[it] = prune(n, tau, cnt);
  }
  return cnt;
}

// One lane per slot (both b2), for s = 64 where a group fills a wavefront.
template <bool ACC>
__device__ __forceinline__ unsigned step_slot(const Matrix& m, Slots in, Slots out, int32_t mode, double tau,
                                              double2* yacc, double coef, int64_t it, int64_t first) {
  const double2 x0 = in.R[2 * it], x1 = in.R[2 * it + 1];
  const double2 y0 = in.Q[2 * it], y1 = in.Q[2 * it + 1];
  const int colq = m.col[it];
  const double v = m.val[it];
  const int pr = m.rev[it];
  const Item x = item_of(m, it, first);
  const Rot r = rotation(v, x.j, colq);
  double2 o0 = x0, o1 = x1, n0 = y0, n1 = y1;
  if (mode == kStep) {
    const double2 c = group_sum(cadd(cjmul(r.f, x0), cscale(x1, r.g)), x.I.s);
    if (ACC && x.live && x.l == 0) {
      double2 yv = yacc[x.I.jbase + x.j];
      yv.x += coef * (c.x * x.I.inv_sqrt_s);
      yv.y += coef * (c.y * x.I.inv_sqrt_s);
      yacc[x.I.jbase + x.j] = yv;
    }
    const double2 tc = cscale(c, 2.0 / double(x.I.s));
    o0 = csub(cmul(tc, r.f), x0);
    o1 = csub(cscale(tc, r.g), x1);
    n0 = cneg(y0);
    n1 = cneg(y1);
  }
  unsigned cnt = 0;
  if (!x.live) return 0;
  o0 = prune(o0, tau, cnt);
  o1 = prune(o1, tau, cnt);
  n1 = prune(n1, tau, cnt);
  if (pr < 0) n0 = prune(n0, tau, cnt);
  write_slot(out, x, it, colq, pr, o0, o1, n0, n1);
  return cnt;
}

// LPS: lanes per slot (2 when every s <= 32, else 1).
template <bool ACC, int LPS>
__device__ __forceinline__ void step_body(StepArgs a) {
  __shared__ unsigned long long sh[16];
  const int64_t A = a.m.items * LPS;
  const int64_t total = A + ((int64_t(a.L.cnt) + kWave - 1) & ~int64_t(kWave - 1));
  double coef = 0.0;
  uint32_t stepno = 0;
  if (ACC) {
    stepno = a.stepno[blockIdx.x];
    coef = a.coefm[stepno];
  }
  unsigned cnt = 0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int lane = threadIdx.x & (kWave - 1);
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < total; it += stride) {
    if (it < A) {
      if (LPS == 2)
        cnt += step_pairs<ACC>(a.m, a.in, a.out, a.mode, a.tau, a.yacc, coef, it, (it - lane) >> 1);
      else
        cnt += step_slot<ACC>(a.m, a.in, a.out, a.mode, a.tau, a.yacc, coef, it, it - lane);
    } else {
      const int64_t e = it - A;
      if (e < int64_t(a.L.cnt)) {
        double2 v = a.L.amp[e];
        if (a.mode == kStep) v = cneg(v);
        a.L.amp[e] = v;
        a.L.key[e] = swap_halves(a.L.key[e], a.m.nbits);
        cnt += nonzero(v);
      }
    }
  }
  const unsigned long long t = block_sum_u64(cnt, sh);
  if (threadIdx.x == 0) {
    atomicAdd(&a.acc[blockIdx.x], t);  // per-workgroup counter: no contention, no return value
    if (ACC) a.stepno[blockIdx.x] = stepno + 1;
  }
}

}  // namespace qw

extern "C" __global__ void __launch_bounds__(256) qwk_step2(qw::StepArgs a) { qw::step_body<false, 2>(a); }
extern "C" __global__ void __launch_bounds__(256) qwk_step2_acc(qw::StepArgs a) { qw::step_body<true, 2>(a); }
extern "C" __global__ void __launch_bounds__(256) qwk_step1(qw::StepArgs a) { qw::step_body<false, 1>(a); }
extern "C" __global__ void __launch_bounds__(256) qwk_step1_acc(qw::StepArgs a) { qw::step_body<true, 1>(a); }

namespace qw {

// ----------------------------------------------------------------- QBS table
// rev[q] = i_{col[q]}(j): where row j's slot q points back into its column's
// row, or -1 (filler or asymmetric pattern).

extern "C" __global__ void __launch_bounds__(256) qwk_qbs_table(Matrix m, int32_t* rev, SlotRec* rec) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < m.items; it += stride) {
    const int ii = find_inst(m, it);
    const Inst I = m.inst[ii];
    const int64_t local = it - I.item_base;
    int32_t r = -1;
    if (local < int64_t(I.N) * I.s) {
      const int j = int(local >> I.hbits);
      const int c = m.col[it];
      int p;
      if (qbs(m.col + I.item_base + int64_t(c) * I.s, I.s, j, p)) r = p;
    }
    rev[it] = r;
    SlotRec sr;
    sr.col = m.col[it];
    sr.rev = r;
    sr.val = m.val[it];
    rec[it] = sr;
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
// of step t.

extern "C" __global__ void __launch_bounds__(256) qwk_adjoint(AdjArgs a) {
  __shared__ unsigned long long sh[16];
  const int n = a.m.nbits;
  const int64_t A = a.m.items;
  const int64_t padL = (int64_t(a.L.cnt) + kWave - 1) & ~int64_t(kWave - 1);
  const int64_t padLL = (int64_t(a.LL.cnt) + kWave - 1) & ~int64_t(kWave - 1);
  const int64_t total = A + padL + padLL;
  unsigned cnt = 0, lcnt = 0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < total; it += stride) {
    if (it < A) {
      const Item x = item_of(a.m, it, it - (threadIdx.x & (kWave - 1)));
      double2 x0 = zero2(), x1 = zero2(), m0 = zero2(), m1 = zero2();
      double2 y0 = zero2(), y1 = zero2(), z0 = zero2(), z1 = zero2();
      Rot r, d;
      r.f = zero2();
      r.g = 0.0;
      d = r;
      int colq = 0, pr = -1;
      if (x.live) {
        x0 = a.in.R[2 * it];
        x1 = a.in.R[2 * it + 1];
        m0 = a.lin.R[2 * it];
        m1 = a.lin.R[2 * it + 1];
        y1 = a.in.Q[2 * it + 1];
        z1 = a.lin.Q[2 * it + 1];
        colq = a.m.col[it];
        pr = a.m.rev[it];
        if (pr < 0) {
          y0 = a.in.Q[2 * it];
          z0 = a.lin.Q[2 * it];
        }
        const double v = a.m.val[it];
        r = rotation(v, x.j, colq);
        d = rotation_deriv(v, x.j, colq);
      }
      const double2 c = group_sum(cadd(cjmul(r.f, x0), cscale(x1, r.g)), x.I.s);
      const double2 dd = group_sum(cadd(cjmul(r.f, m0), cscale(m1, r.g)), x.I.s);
      const double t = 2.0 / double(x.I.s);
      const double2 tc = cscale(c, t), td = cscale(dd, t);
      double2 q0 = csub(cmul(tc, r.f), x0);  // psi'
      double2 q1 = csub(cscale(tc, r.g), x1);
      double2 w0 = csub(cmul(td, r.f), m0);  // reflected adjoint
      double2 w1 = csub(cscale(td, r.g), m1);
      if (x.live) {
        // c (conj(mu_0) f' + conj(mu_1) g') + conj(d) (conj(f') psi'_0 + g' psi'_1)
        const double2 u = cadd(cmul(c, cadd(cjmul(m0, d.f), make_double2(m1.x * d.g, -m1.y * d.g))),
                               cjmul(dd, cadd(cjmul(d.f, q0), cscale(q1, d.g))));
        a.dv[it] += 2.0 * t * u.x;
        q0 = prune(q0, a.tau, cnt);
        q1 = prune(q1, a.tau, cnt);
        const double2 ny1 = prune(cneg(y1), a.tau, cnt);
        const double2 ny0 = pr < 0 ? prune(cneg(y0), a.tau, cnt) : zero2();
        write_slot(a.out, x, it, colq, pr, q0, q1, ny0, ny1);
        w0 = prune(w0, a.tau, lcnt);
        w1 = prune(w1, a.tau, lcnt);
        const double2 nz1 = prune(cneg(z1), a.tau, lcnt);
        const double2 nz0 = pr < 0 ? prune(cneg(z0), a.tau, lcnt) : zero2();
        write_slot(a.lout, x, it, colq, pr, w0, w1, nz0, nz1);
      }
    } else {
      const bool second = it >= A + padL;
      const int64_t e = second ? it - A - padL : it - A;
      const List& Ls = second ? a.LL : a.L;
      if (e < int64_t(Ls.cnt)) {
        const double2 v = cneg(Ls.amp[e]);
        Ls.amp[e] = v;
        Ls.key[e] = swap_halves(Ls.key[e], n);
        (second ? lcnt : cnt) += nonzero(v);
      }
    }
  }
  const unsigned long long t1 = block_sum_u64(cnt, sh);
  if (threadIdx.x == 0) a.acc[blockIdx.x] += t1;
  const unsigned long long t2 = block_sum_u64(lcnt, sh);
  if (threadIdx.x == 0) a.lacc[blockIdx.x] += t2;
}

// ----------------------------------------------------------------- T~ |b~>
// T~ on |0, j, 0, 0, 0, 0> gives the group of j with amplitudes b_j phi_j:
// slot (j, l) receives b_j f/sqrt(s) and b_j g/sqrt(s) (Alg. 5).

extern "C" __global__ void __launch_bounds__(256) qwk_init(Matrix m, const double2* __restrict__ b, Slots out,
                                                           double tau) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < m.items; it += stride) {
    const int ii = find_inst(m, it);
    const Inst I = m.inst[ii];
    const int64_t local = it - I.item_base;
    if (local >= int64_t(I.N) * I.s) continue;
    const int j = int(local >> I.hbits);
    const Rot r = rotation(m.val[it], j, m.col[it]);
    const double2 bj = cscale(b[I.jbase + j], I.inv_sqrt_s);
    double2 o0 = cmul(r.f, bj);
    double2 o1 = cscale(bj, r.g);
    if (!kept(o0, tau)) o0 = zero2();
    if (!kept(o1, tau)) o1 = zero2();
    out.R[2 * it] = o0;
    out.R[2 * it + 1] = o1;
  }
}

// ----------------------------------------------------------------- fill (zero)

extern "C" __global__ void qwk_fill(uint4* p, int64_t n16) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// ----------------------------------------------------------------- measurements

// kind 0: count, 1: norm^2 -> partial[block]; kind 2: j marginal (atomics
// into out, which starts at zero); kind 3: projection (stored).
extern "C" __global__ void __launch_bounds__(256) qwk_measure(Matrix m, Slots st, List L, int32_t kind,
                                                              double* partial, double* out) {
  __shared__ double sh[16];
  const int n = m.nbits;
  const uint64_t nm = (uint64_t(1) << n) - 1;
  const int64_t total = m.items + ((int64_t(L.cnt) + kWave - 1) & ~int64_t(kWave - 1));
  double acc = 0.0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < total; it += stride) {
    if (it < m.items) {
      const Item x = item_of(m, it, it - (threadIdx.x & (kWave - 1)));
      double2 p0 = zero2(), p1 = zero2(), s0 = zero2(), s1 = zero2();
      int colq = 0;
      if (x.live) {
        p0 = st.R[2 * it];
        p1 = st.R[2 * it + 1];
        s0 = st.Q[2 * it];
        s1 = st.Q[2 * it + 1];
        colq = m.col[it];
      }
      if (kind == 0) {
        acc += double(int(nonzero(p0)) + int(nonzero(p1)) + int(nonzero(s0)) + int(nonzero(s1)));
      } else if (kind == 1) {
        acc += p0.x * p0.x + p0.y * p0.y + p1.x * p1.x + p1.y * p1.y + s0.x * s0.x + s0.y * s0.y + s1.x * s1.x +
               s1.y * s1.y;
      } else if (kind == 2) {
        double2 q = make_double2(p0.x * p0.x + p0.y * p0.y + p1.x * p1.x + p1.y * p1.y, 0.0);
        q = group_sum(q, x.I.s);
        if (x.live) {
          if (x.l == 0) atomicAdd(&out[x.I.jbase + x.j], q.x);
          const double sw = s0.x * s0.x + s0.y * s0.y + s1.x * s1.x + s1.y * s1.y;
          if (sw != 0.0) atomicAdd(&out[x.I.jbase + colq], sw);
        }
      } else {
        Rot r;
        r.f = zero2();
        r.g = 0.0;
        if (x.live) r = rotation(m.val[it], x.j, colq);
        const double2 c = group_sum(cadd(cjmul(r.f, p0), cscale(p1, r.g)), x.I.s);
        if (x.live && x.l == 0) {
          out[2 * (x.I.jbase + x.j)] = c.x * x.I.inv_sqrt_s;
          out[2 * (x.I.jbase + x.j) + 1] = c.y * x.I.inv_sqrt_s;
        }
      }
    } else {
      const int64_t e = it - m.items;
      if (e < int64_t(L.cnt)) {
        const double2 v = L.amp[e];
        if (kind == 0) {
          acc += double(nonzero(v));
        } else if (kind == 1) {
          acc += v.x * v.x + v.y * v.y;
        } else if (kind == 2) {
          const uint64_t key = L.key[e];
          const uint64_t inst = key >> (4 * n + 2);
          const int j = int((key >> (2 * n + 2)) & nm);
          if (inst < uint64_t(m.ninst)) atomicAdd(&out[m.inst[inst].jbase + j], v.x * v.x + v.y * v.y);
        }
      }
    }
  }
  if (kind <= 1) {
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
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
      const Item x = item_of(m, it, it - (threadIdx.x & (kWave - 1)));
      if (x.live) {
        const int colq = m.col[it];
        for (int b2 = 0; b2 < 2; ++b2) {
          v[b2] = st.R[2 * it + b2];
          app[b2] = nonzero(v[b2]);
          k[b2] = member_key(uint64_t(x.inst), n, x.j, colq, b2);
          v[2 + b2] = st.Q[2 * it + b2];
          app[2 + b2] = nonzero(v[2 + b2]);
          k[2 + b2] = swapped_key(uint64_t(x.inst), n, x.j, colq, b2);
        }
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

// Home of a key: 0 = R (group member), 1 = Q (swap of a member), 2 = list.
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
  if (jc != 0 || kc != 0 || inst >= uint64_t(m.ninst)) return 2;
  const Inst I = m.inst[inst];
  if (j >= I.N || k >= I.N) return 2;
  int p;
  if (b1 == 0 && qbs(m.col + I.item_base + int64_t(j) * I.s, I.s, k, p)) {
    idx = 2 * (I.item_base + int64_t(j) * I.s + p) + b2;
    return 0;
  }
  // (0, J, B1, 0, K, 0) = S K(q, B1) with q = (K, position of J in row K)
  if (b2 == 0 && qbs(m.col + I.item_base + int64_t(k) * I.s, I.s, j, p)) {
    idx = 2 * (I.item_base + int64_t(k) * I.s + p) + b1;
    return 1;
  }
  return 2;
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
        out.R[idx] = v[0];
      else if (h == 1)
        out.Q[idx] = v[0];
      else
        app[0] = true;
    }
    wave_append4(L.key, L.amp, lcnt, L.cap, app, k, v);
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
      const Item x = item_of(m, it, it - (threadIdx.x & (kWave - 1)));
      if (x.live) {
        const double wr = w[x.I.jbase + m.col[it]];
        const double wq = w[x.I.jbase + x.j];
        for (int b2 = 0; b2 < 2; ++b2) {
          const double2 p = in.R[2 * it + b2];
          const double2 s = in.Q[2 * it + b2];
          acc += wr * (p.x * p.x + p.y * p.y) + wq * (s.x * s.x + s.y * s.y);
          out.R[2 * it + b2] = cscale(p, wr);
          out.Q[2 * it + b2] = cscale(s, wq);
        }
      }
    } else {
      const int64_t e = it - m.items;
      if (e < int64_t(L.cnt)) {
        const uint64_t key = L.key[e];
        const double2 p = L.amp[e];
        const uint64_t inst = key >> (4 * n + 2);
        const int k = int((key >> 1) & nm);
        const double wk = inst < uint64_t(m.ninst) ? w[m.inst[inst].jbase + k] : 0.0;
        acc += wk * (p.x * p.x + p.y * p.y);
        LL.key[e] = key;
        LL.amp[e] = cscale(p, wk);
      }
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Gradient through the initial T~: psi_0 holds b_j phi_j in the group of j,
// so dL/dv_{jl} += 2 Re[b_j (conj(nu_0) f' + conj(nu_1) g')] / sqrt(s) with
// nu the group amplitudes of lambda_0, and dL/db_j = 2 <psi~_j|lambda_0>.
extern "C" __global__ void __launch_bounds__(256) qwk_grad_init(Matrix m, Slots lam, const double2* b, double* dv,
                                                                double2* db) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < m.items; it += stride) {
    const Item x = item_of(m, it, it - (threadIdx.x & (kWave - 1)));
    double2 n0 = zero2(), n1 = zero2();
    Rot r, d;
    r.f = zero2();
    r.g = 0.0;
    d = r;
    if (x.live) {
      n0 = lam.R[2 * it];
      n1 = lam.R[2 * it + 1];
      const int colq = m.col[it];
      const double v = m.val[it];
      r = rotation(v, x.j, colq);
      d = rotation_deriv(v, x.j, colq);
      const double2 bj = b[x.I.jbase + x.j];
      const double2 u = cmul(bj, cadd(cjmul(n0, d.f), make_double2(n1.x * d.g, -n1.y * d.g)));
      dv[it] += 2.0 * u.x * x.I.inv_sqrt_s;
    }
    const double2 c = group_sum(cadd(cjmul(r.f, n0), cscale(n1, r.g)), x.I.s);
    if (x.live && x.l == 0) db[x.I.jbase + x.j] = cscale(c, 2.0 * x.I.inv_sqrt_s);
  }
}

}  // namespace qw
