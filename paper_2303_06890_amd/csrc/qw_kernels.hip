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
// keys, so the only interference in a step is one reduction per group j; no
// global sort is needed.  The group of j is exactly the set of keys
// (0, j, 0, 0, k_{j,l}, b2), l < s: it has a fixed address, the ELL slot
// (j, l).  A state is therefore held as
//   R[2q + b2]  amplitude of key (0, j, 0, 0, col[q], b2) for ELL slot q=(j,l)
//   a list      (key, amplitude) of every other branch (structure of arrays)
// and one kernel per step does, for every slot q (phase A): read the pair,
// reduce c_j = sum_l conj(f) psi(l,0) + g psi(l,1) over the s lanes of the
// group (wave shuffles), write 2c_j phi - psi, apply S, and send each output
// branch to its home for the next step (a slot when the output key is a group
// member, found with the quantum binary search of the row; else a list
// append compacted with wave ballots and one atomic per wave); and for every
// list entry (phase B): negate, apply S, send home.  Branches with |Re| and
// |Im| <= tau are dropped on output.  The consumed R entries are zeroed as
// they are read, so the two R buffers alternate without a clearing pass.
#include "qw_internal.h"

#include <hip/hip_runtime.h>

namespace qw {

static_assert(sizeof(Ctl) == 512, "control block layout");

// ----------------------------------------------------------------- helpers

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double t) { return make_double2(a.x * t, a.y * t); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 cjmul(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ bool nonzero_tau(double2 v, double tau) { return fabs(v.x) > tau || fabs(v.y) > tau; }

// Rotation amplitudes of Sec. IV (footnote on negative elements):
// f = sqrt(a) for a >= 0, +-i sqrt|a| (+ when row j <= column k) for a < 0,
// g = sqrt(1 - |a|).
struct Rot {
  double2 f;
  double g;
};
__device__ __forceinline__ Rot rotation(double a, int j, int k) {
  Rot r;
  if (a >= 0.0) {
    r.f = make_double2(sqrt(a), 0.0);
  } else {
    const double q = sqrt(-a);
    r.f = make_double2(0.0, j <= k ? q : -q);
  }
  r.g = sqrt(1.0 - fabs(a));
  return r;
}
// d f/da and d g/da (not finite at a = 0 and |a| = 1).
__device__ __forceinline__ Rot rotation_deriv(double a, int j, int k) {
  Rot d;
  if (a > 0.0) {
    d.f = make_double2(0.5 / sqrt(a), 0.0);
  } else if (a < 0.0) {
    const double q = -0.5 / sqrt(-a);
    d.f = make_double2(0.0, j <= k ? q : -q);
  } else {
    d.f = make_double2(__builtin_inf(), 0.0);
  }
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

// Sum over aligned groups of `width` lanes (width a power of two <= 64).
// Every lane of a group ends with the bitwise-identical sum.
__device__ __forceinline__ double2 group_sum(double2 v, int width) {
  for (int off = 1; off < width; off <<= 1) {
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

// Key of the slot entry (0, j, 0, 0, col, b2) of instance `inst`.
__device__ __forceinline__ uint64_t slot_key(uint64_t inst, int n, int j, int col, int b2) {
  return (inst << (4 * n + 2)) | (uint64_t(j) << (2 * n + 2)) | (uint64_t(col) << 1) | uint64_t(b2);
}

// Home of a branch for the next step: if the key is a group member
// (j_c = b1 = k_c = 0 and k in row j) return true and its slot index.
__device__ __forceinline__ bool home_slot(const Matrix& m, uint64_t key, int64_t& slot, int& b2) {
  const int n = m.nbits;
  const uint64_t nm = (uint64_t(1) << n) - 1;
  b2 = int(key & 1);
  const int k = int((key >> 1) & nm);
  const uint64_t kc = (key >> (n + 1)) & nm;
  const uint64_t b1 = (key >> (2 * n + 1)) & 1;
  const int j = int((key >> (2 * n + 2)) & nm);
  const uint64_t jc = (key >> (3 * n + 2)) & nm;
  const uint64_t inst = key >> (4 * n + 2);
  if (jc != 0 || b1 != 0 || kc != 0 || inst >= uint64_t(m.ninst)) return false;
  const Inst I = m.inst[inst];
  if (j >= I.N || k >= I.N) return false;
  const int64_t row = I.item_base + int64_t(j) * I.s;
  int p;
  if (!qbs(m.col + row, I.s, k, p)) return false;
  slot = row + p;
  return true;
}

// Wave-level compacted append of up to two values per lane to a list.
__device__ __forceinline__ void wave_append(const Buf& out, uint32_t cap, bool app0, uint64_t k0, double2 v0,
                                            bool app1, uint64_t k1, double2 v1, bool& overflow) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  const uint64_t m0 = __ballot(app0);
  const uint64_t m1 = __ballot(app1);
  const uint32_t n0 = __popcll(m0), n1 = __popcll(m1);
  if (n0 + n1 == 0) return;
  uint32_t base = 0;
  if (lane == 0) base = atomicAdd(out.cnt, n0 + n1);
  base = __shfl(base, 0);
  if (app0) {
    const uint32_t idx = base + __popcll(m0 & lt);
    if (idx < cap) {
      out.key[idx] = k0;
      out.amp[idx] = v0;
    } else {
      overflow = true;
    }
  }
  if (app1) {
    const uint32_t idx = base + n0 + __popcll(m1 & lt);
    if (idx < cap) {
      out.key[idx] = k1;
      out.amp[idx] = v1;
    } else {
      overflow = true;
    }
  }
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Last-workgroup bookkeeping: the input list has been consumed, counters
// advance.  Called by every thread after its work.
__device__ __forceinline__ void finish_launch(Ctl* ctl, uint32_t* in_cnt, unsigned long long kept, bool overflow) {
  const int lane = threadIdx.x & (kWave - 1);
  kept = wave_sum_u64(kept);
  const bool any_over = __ballot(overflow) != 0;
  if (lane == 0) {
    if (kept) atomicAdd(&ctl->written, kept);
    if (any_over) atomicOr(&ctl->overflow, 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t ticket = atomicAdd(&ctl->done, 1u);
    if (ticket == gridDim.x - 1) {
      __threadfence();
      *in_cnt = 0;
      ctl->done = 0;
      const unsigned long long w = atomicExch(&ctl->written, 0ull);
      ctl->last_written = w;
      ctl->total_written += w;
      ctl->steps += 1;
      ctl->stepno += 1;
      __threadfence();
    }
  }
}

// ----------------------------------------------------------------- walk step

template <bool ACC>
__device__ __forceinline__ void step_body(StepArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int n = a.m.nbits;
  const int64_t A = a.m.items;
  const uint32_t B = min(*a.in.cnt, a.in.cap);
  const int64_t total = A + ((int64_t(B) + kWave - 1) & ~int64_t(kWave - 1));
  double coef = 0.0;
  if (ACC) coef = a.coefm[a.ctl->stepno];
  const bool reflect = a.mode == kStep;
  unsigned long long kept = 0;
  bool overflow = false;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < total; it += stride) {
    bool app0 = false, app1 = false;
    uint64_t k0 = 0, k1 = 0;
    double2 v0 = make_double2(0.0, 0.0), v1 = v0;
    if (it < A) {
      // ---- phase A: one ELL slot (j, l) per lane, a group of s lanes per row j
      const int ii = __builtin_amdgcn_readfirstlane(find_inst(a.m, it - lane));
      const Inst I = a.m.inst[ii];
      const int64_t local = it - I.item_base;
      const bool live = local < int64_t(I.N) * I.s;
      const int l = int(local) & (I.s - 1);
      const int j = int(local >> I.hbits);
      double2 p0 = make_double2(0.0, 0.0), p1 = p0;
      Rot r;
      r.f = p0;
      r.g = 0.0;
      int colq = 0;
      if (live) {
        p0 = a.in.R[2 * it];
        p1 = a.in.R[2 * it + 1];
        a.in.R[2 * it] = make_double2(0.0, 0.0);
        a.in.R[2 * it + 1] = make_double2(0.0, 0.0);
        colq = a.m.col[it];
        r = rotation(a.m.val[it], j, colq);
      }
      double2 o0 = p0, o1 = p1;
      if (reflect) {
        double2 c = cadd(cjmul(r.f, p0), cscale(p1, r.g));
        c = group_sum(c, I.s);
        if (ACC && live && l == 0) {
          double2 y = a.yacc[I.jbase + j];
          y.x += coef * (c.x * I.inv_sqrt_s);
          y.y += coef * (c.y * I.inv_sqrt_s);
          a.yacc[I.jbase + j] = y;
        }
        const double2 tc = cscale(c, 2.0 / double(I.s));
        o0 = csub(cmul(tc, r.f), p0);
        o1 = csub(cscale(tc, r.g), p1);
      }
      const bool keep0 = live && nonzero_tau(o0, a.tau);
      const bool keep1 = live && nonzero_tau(o1, a.tau);
      // after S the keys are (0, col, b2, 0, j, 0)
      k0 = (uint64_t(ii) << (4 * n + 2)) | (uint64_t(colq) << (2 * n + 2)) | (uint64_t(j) << 1);
      k1 = k0 | (uint64_t(1) << (2 * n + 1));
      if (keep0) {
        int p;
        if (qbs(a.m.col + I.item_base + int64_t(colq) * I.s, I.s, j, p)) {
          a.out.R[2 * (I.item_base + int64_t(colq) * I.s + p)] = o0;
        } else {
          app0 = true;
          v0 = o0;
        }
      }
      if (keep1) {
        app1 = true;
        v1 = o1;
      }
      kept += unsigned(keep0) + unsigned(keep1);
    } else {
      // ---- phase B: one list entry per lane; P R H P H R^dagger = -1 there
      const int64_t e = it - A;
      if (e < int64_t(B)) {
        const uint64_t key = a.in.key[e];
        double2 v = a.in.amp[e];
        if (reflect) v = make_double2(-v.x, -v.y);
        if (nonzero_tau(v, a.tau)) {
          ++kept;
          const uint64_t kk = swap_halves(key, n);
          int64_t slot;
          int b2;
          if (home_slot(a.m, kk, slot, b2)) {
            a.out.R[2 * slot + b2] = v;
          } else {
            app0 = true;
            k0 = kk;
            v0 = v;
          }
        }
      }
    }
    wave_append(a.out, a.cap, app0, k0, v0, app1, k1, v1, overflow);
  }
  finish_launch(a.ctl, a.in.cnt, kept, overflow);
}

}  // namespace qw

extern "C" __global__ void __launch_bounds__(256) qwk_step(qw::StepArgs a) { qw::step_body<false>(a); }
extern "C" __global__ void __launch_bounds__(256) qwk_step_acc(qw::StepArgs a) { qw::step_body<true>(a); }

namespace qw {


// ----------------------------------------------------------------- adjoint sweep step
// One reverse step of the gradient: both the recomputed state Psi_t and the
// adjoint state Lambda_t (each kept S-conjugated, so that W^dagger acts as W)
// advance by one walk step, and every slot (j, l) accumulates
//   dL/dv_{jl} += 2 Re[ (2/s) ( c (conj(mu_0) f' + conj(mu_1) g')
//                              + conj(d) (conj(f') psi'_0 + g' psi'_1) ) ]
// where chi, mu are the slot amplitudes of Psi_t and Lambda_t, c, d their
// group sums, and psi' = (2/s) c phi - chi the forward state before the
// reflection of step t.

extern "C" __global__ void __launch_bounds__(256) qwk_adjoint(AdjArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int n = a.m.nbits;
  const int64_t A = a.m.items;
  const uint32_t B = min(*a.in.cnt, a.in.cap);
  const uint32_t BL = min(*a.lin.cnt, a.lin.cap);
  const int64_t padB = (int64_t(B) + kWave - 1) & ~int64_t(kWave - 1);
  const int64_t padBL = (int64_t(BL) + kWave - 1) & ~int64_t(kWave - 1);
  const int64_t total = A + padB + padBL;
  unsigned long long kept = 0, lkept = 0;
  bool overflow = false, loverflow = false;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < total; it += stride) {
    if (it < A) {
      const int ii = __builtin_amdgcn_readfirstlane(find_inst(a.m, it - lane));
      const Inst I = a.m.inst[ii];
      const int64_t local = it - I.item_base;
      const bool live = local < int64_t(I.N) * I.s;
      const int l = int(local) & (I.s - 1);
      const int j = int(local >> I.hbits);
      double2 x0 = make_double2(0.0, 0.0), x1 = x0, m0 = x0, m1 = x0;
      Rot r, d;
      r.f = x0;
      r.g = 0.0;
      d = r;
      int colq = 0;
      if (live) {
        x0 = a.in.R[2 * it];
        x1 = a.in.R[2 * it + 1];
        m0 = a.lin.R[2 * it];
        m1 = a.lin.R[2 * it + 1];
        a.in.R[2 * it] = make_double2(0.0, 0.0);
        a.in.R[2 * it + 1] = make_double2(0.0, 0.0);
        a.lin.R[2 * it] = make_double2(0.0, 0.0);
        a.lin.R[2 * it + 1] = make_double2(0.0, 0.0);
        colq = a.m.col[it];
        const double v = a.m.val[it];
        r = rotation(v, j, colq);
        d = rotation_deriv(v, j, colq);
      }
      const double2 c = group_sum(cadd(cjmul(r.f, x0), cscale(x1, r.g)), I.s);
      const double2 dd = group_sum(cadd(cjmul(r.f, m0), cscale(m1, r.g)), I.s);
      const double t = 2.0 / double(I.s);
      const double2 tc = cscale(c, t), td = cscale(dd, t);
      const double2 q0 = csub(cmul(tc, r.f), x0);  // psi'
      const double2 q1 = csub(cscale(tc, r.g), x1);
      const double2 w0 = csub(cmul(td, r.f), m0);  // reflected adjoint
      const double2 w1 = csub(cscale(td, r.g), m1);
      if (live) {
        // c (conj(mu_0) f' + conj(mu_1) g') + conj(d) (conj(f') psi'_0 + g' psi'_1)
        const double2 u = cadd(cmul(c, cadd(cjmul(m0, d.f), make_double2(m1.x * d.g, -m1.y * d.g))),
                               cjmul(dd, cadd(cjmul(d.f, q0), cscale(q1, d.g))));
        a.dv[it] += 2.0 * t * u.x;
      }
      const uint64_t kbase = (uint64_t(ii) << (4 * n + 2)) | (uint64_t(colq) << (2 * n + 2)) | (uint64_t(j) << 1);
      const uint64_t kb1 = kbase | (uint64_t(1) << (2 * n + 1));
      int p = 0;
      const bool found = live && qbs(a.m.col + I.item_base + int64_t(colq) * I.s, I.s, j, p);
      const int64_t dst = 2 * (I.item_base + int64_t(colq) * I.s + p);
      // recomputed state
      {
        const bool keep0 = live && nonzero_tau(q0, a.tau);
        const bool keep1 = live && nonzero_tau(q1, a.tau);
        bool app0 = false;
        if (keep0) {
          if (found)
            a.out.R[dst] = q0;
          else
            app0 = true;
        }
        kept += unsigned(keep0) + unsigned(keep1);
        wave_append(a.out, a.cap, app0, kbase, q0, keep1, kb1, q1, overflow);
      }
      // adjoint state
      {
        const bool keep0 = live && nonzero_tau(w0, a.tau);
        const bool keep1 = live && nonzero_tau(w1, a.tau);
        bool app0 = false;
        if (keep0) {
          if (found)
            a.lout.R[dst] = w0;
          else
            app0 = true;
        }
        lkept += unsigned(keep0) + unsigned(keep1);
        wave_append(a.lout, a.cap, app0, kbase, w0, keep1, kb1, w1, loverflow);
      }
    } else {
      const bool second = it >= A + padB;
      const int64_t e = second ? it - A - padB : it - A;
      const Buf& src = second ? a.lin : a.in;
      const Buf& dst = second ? a.lout : a.out;
      const uint32_t cnt = second ? BL : B;
      bool app = false;
      uint64_t kk = 0;
      double2 v = make_double2(0.0, 0.0);
      if (e < int64_t(cnt)) {
        v = src.amp[e];
        v = make_double2(-v.x, -v.y);
        if (nonzero_tau(v, a.tau)) {
          (second ? lkept : kept) += 1;
          kk = swap_halves(src.key[e], n);
          int64_t slot;
          int b2;
          if (home_slot(a.m, kk, slot, b2))
            dst.R[2 * slot + b2] = v;
          else
            app = true;
        }
      }
      // `second` is wave-uniform (the list ranges are wave aligned)
      wave_append(dst, a.cap, app, kk, v, false, 0, v, second ? loverflow : overflow);
    }
  }
  finish_launch(a.lctl, a.lin.cnt, lkept, loverflow);
  finish_launch(a.ctl, a.in.cnt, kept, overflow);
}


// ----------------------------------------------------------------- T~ |b~>
// T~ on |0, j, 0, 0, 0, 0> gives the group of j with amplitudes b_j phi_j:
// slot (j, l) receives b_j f/sqrt(s) and b_j g/sqrt(s) (Alg. 5).

extern "C" __global__ void __launch_bounds__(256) qwk_init(Matrix m, const double2* __restrict__ b, Buf out, double tau) {
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
    if (!nonzero_tau(o0, tau)) o0 = make_double2(0.0, 0.0);
    if (!nonzero_tau(o1, tau)) o1 = make_double2(0.0, 0.0);
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

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < int(blockDim.x >> 6); ++i) t += sh[i];
  return t;
}

// kind 0: count, 1: norm^2 -> partial[block]; kind 2: j marginal (R part
// stored, list part added atomically); kind 3: projection.
extern "C" __global__ void __launch_bounds__(256) qwk_measure(Matrix m, Buf b, int32_t kind, double* partial, double* out) {
  __shared__ double sh[16];
  const int lane = threadIdx.x & (kWave - 1);
  const int n = m.nbits;
  const uint32_t B = min(*b.cnt, b.cap);
  const int64_t padA = m.items;
  const int64_t total = padA + ((int64_t(B) + kWave - 1) & ~int64_t(kWave - 1));
  double acc = 0.0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < total; it += stride) {
    if (it < padA) {
      const int ii = __builtin_amdgcn_readfirstlane(find_inst(m, it - lane));
      const Inst I = m.inst[ii];
      const int64_t local = it - I.item_base;
      const bool live = local < int64_t(I.N) * I.s;
      const int l = int(local) & (I.s - 1);
      const int j = int(local >> I.hbits);
      double2 p0 = make_double2(0.0, 0.0), p1 = p0;
      if (live) {
        p0 = b.R[2 * it];
        p1 = b.R[2 * it + 1];
      }
      if (kind == 0) {
        acc += double((p0.x != 0.0 || p0.y != 0.0) + (p1.x != 0.0 || p1.y != 0.0));
      } else if (kind == 1) {
        acc += p0.x * p0.x + p0.y * p0.y + p1.x * p1.x + p1.y * p1.y;
      } else if (kind == 2) {
        double2 q = make_double2(p0.x * p0.x + p0.y * p0.y + p1.x * p1.x + p1.y * p1.y, 0.0);
        q = group_sum(q, I.s);
        if (live && l == 0) out[I.jbase + j] = q.x;
      } else {
        Rot r;
        r.f = make_double2(0.0, 0.0);
        r.g = 0.0;
        if (live) r = rotation(m.val[it], j, m.col[it]);
        double2 c = group_sum(cadd(cjmul(r.f, p0), cscale(p1, r.g)), I.s);
        if (live && l == 0) {
          out[2 * (I.jbase + j)] = c.x * I.inv_sqrt_s;
          out[2 * (I.jbase + j) + 1] = c.y * I.inv_sqrt_s;
        }
      }
    } else if (kind <= 1) {
      const int64_t e = it - padA;
      if (e < int64_t(B)) {
        const double2 v = b.amp[e];
        acc += kind == 0 ? 1.0 : v.x * v.x + v.y * v.y;
      }
    }
  }
  if (kind <= 1) {
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
  }
}

// list part of the j marginal
extern "C" __global__ void __launch_bounds__(256) qwk_marginal_list(Matrix m, Buf b, double* out) {
  const int n = m.nbits;
  const uint64_t nm = (uint64_t(1) << n) - 1;
  const uint32_t B = min(*b.cnt, b.cap);
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < int64_t(B); e += stride) {
    const uint64_t key = b.key[e];
    const double2 v = b.amp[e];
    const uint64_t inst = key >> (4 * n + 2);
    if (inst >= uint64_t(m.ninst)) continue;
    const int j = int((key >> (2 * n + 2)) & nm);
    atomicAdd(&out[m.inst[inst].jbase + j], v.x * v.x + v.y * v.y);
  }
}


// ----------------------------------------------------------------- export / import

extern "C" __global__ void __launch_bounds__(256) qwk_export(Matrix m, Buf b, uint64_t* keys, double2* amps, uint32_t* count,
                                                     uint32_t cap) {
  const int lane = threadIdx.x & (kWave - 1);
  const int n = m.nbits;
  const uint32_t B = min(*b.cnt, b.cap);
  const int64_t total = m.items + ((int64_t(B) + kWave - 1) & ~int64_t(kWave - 1));
  Buf out;
  out.key = keys;
  out.amp = amps;
  out.cnt = count;
  out.cap = cap;
  out.R = nullptr;
  bool overflow = false;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < total; it += stride) {
    bool a0 = false, a1 = false;
    uint64_t k0 = 0, k1 = 0;
    double2 v0 = make_double2(0.0, 0.0), v1 = v0;
    if (it < m.items) {
      const int ii = __builtin_amdgcn_readfirstlane(find_inst(m, it - lane));
      const Inst I = m.inst[ii];
      const int64_t local = it - I.item_base;
      if (local < int64_t(I.N) * I.s) {
        const int j = int(local >> I.hbits);
        const int colq = m.col[it];
        v0 = b.R[2 * it];
        v1 = b.R[2 * it + 1];
        a0 = v0.x != 0.0 || v0.y != 0.0;
        a1 = v1.x != 0.0 || v1.y != 0.0;
        k0 = slot_key(uint64_t(ii), n, j, colq, 0);
        k1 = slot_key(uint64_t(ii), n, j, colq, 1);
      }
    } else {
      const int64_t e = it - m.items;
      if (e < int64_t(B)) {
        a0 = true;
        k0 = b.key[e];
        v0 = b.amp[e];
      }
    }
    wave_append(out, cap, a0, k0, v0, a1, k1, v1, overflow);
  }
}


// Place branches (unique keys, validated on the host) at their homes.
extern "C" __global__ void __launch_bounds__(256) qwk_import(Matrix m, const uint64_t* keys, const double2* amps, int64_t cnt,
                                                     Buf out, Ctl* ctl, uint32_t cap) {
  bool overflow = false;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t total = (cnt + kWave - 1) & ~int64_t(kWave - 1);
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += stride) {
    bool app = false;
    uint64_t key = 0;
    double2 v = make_double2(0.0, 0.0);
    if (e < cnt) {
      key = keys[e];
      v = amps[e];
      int64_t slot;
      int b2;
      if (home_slot(m, key, slot, b2))
        out.R[2 * slot + b2] = v;
      else
        app = true;
    }
    wave_append(out, cap, app, key, v, false, 0, v, overflow);
  }
  if (__ballot(overflow) != 0 && (threadIdx.x & 63) == 0) atomicOr(&ctl->overflow, 1u);
}


// ----------------------------------------------------------------- gradient set-up and finish

// Lambda = diag(w[k register]) Psi for a state kept S-conjugated (the j
// register of the true state is the k register of the stored one), and the
// loss sum_branches w |amp|^2 as per-block partials.
extern "C" __global__ void __launch_bounds__(256) qwk_weight(Matrix m, Buf in, Buf out, const double* w, uint32_t cap,
                                                     double* partial) {
  __shared__ double sh[16];
  const int lane = threadIdx.x & (kWave - 1);
  const int n = m.nbits;
  const uint64_t nm = (uint64_t(1) << n) - 1;
  const uint32_t B = min(*in.cnt, in.cap);
  const int64_t total = m.items + ((int64_t(B) + kWave - 1) & ~int64_t(kWave - 1));
  double acc = 0.0;
  bool overflow = false;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < total; it += stride) {
    bool app = false;
    uint64_t key = 0;
    double2 v = make_double2(0.0, 0.0);
    if (it < m.items) {
      const int ii = __builtin_amdgcn_readfirstlane(find_inst(m, it - lane));
      const Inst I = m.inst[ii];
      const int64_t local = it - I.item_base;
      if (local < int64_t(I.N) * I.s) {
        const double wk = w[I.jbase + m.col[it]];
        const double2 p0 = in.R[2 * it], p1 = in.R[2 * it + 1];
        acc += wk * (p0.x * p0.x + p0.y * p0.y + p1.x * p1.x + p1.y * p1.y);
        out.R[2 * it] = cscale(p0, wk);
        out.R[2 * it + 1] = cscale(p1, wk);
      }
    } else {
      const int64_t e = it - m.items;
      if (e < int64_t(B)) {
        key = in.key[e];
        const double2 p = in.amp[e];
        const uint64_t inst = key >> (4 * n + 2);
        const int k = int((key >> 1) & nm);
        const double wk = inst < uint64_t(m.ninst) ? w[m.inst[inst].jbase + k] : 0.0;
        acc += wk * (p.x * p.x + p.y * p.y);
        v = cscale(p, wk);
        app = wk != 0.0;
      }
    }
    wave_append(out, cap, app, key, v, false, 0, v, overflow);
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}


// Gradient through the initial T~: psi_0 holds b_j phi_j in the group of j,
// so dL/dv_{jl} += 2 Re[b_j (conj(nu_0) f' + conj(nu_1) g')] / sqrt(s) with
// nu the slot amplitudes of lambda_0, and dL/db_j = 2 <psi~_j|lambda_0>.
extern "C" __global__ void __launch_bounds__(256) qwk_grad_init(Matrix m, Buf lam, const double2* b, double* dv, double2* db) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < m.items; it += stride) {
    const int ii = __builtin_amdgcn_readfirstlane(find_inst(m, it - lane));
    const Inst I = m.inst[ii];
    const int64_t local = it - I.item_base;
    const bool live = local < int64_t(I.N) * I.s;
    const int l = int(local) & (I.s - 1);
    const int j = int(local >> I.hbits);
    double2 n0 = make_double2(0.0, 0.0), n1 = n0, bj = n0;
    Rot r, d;
    r.f = n0;
    r.g = 0.0;
    d = r;
    if (live) {
      n0 = lam.R[2 * it];
      n1 = lam.R[2 * it + 1];
      const int colq = m.col[it];
      const double v = m.val[it];
      r = rotation(v, j, colq);
      d = rotation_deriv(v, j, colq);
      bj = b[I.jbase + j];
      const double2 u = cmul(bj, cadd(cjmul(n0, d.f), make_double2(n1.x * d.g, -n1.y * d.g)));
      dv[it] += 2.0 * u.x * I.inv_sqrt_s;
    }
    const double2 c = group_sum(cadd(cjmul(r.f, n0), cscale(n1, r.g)), I.s);
    if (live && l == 0) db[I.jbase + j] = cscale(c, 2.0 * I.inv_sqrt_s);
  }
}


}  // namespace qw
