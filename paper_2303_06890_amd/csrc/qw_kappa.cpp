// Condition number of the walk's matrix on the host: kappa = 1 / min |lambda|
// of A/s (Sec. V.B, preprocessing list: A is rescaled so that its entries lie
// in [-1, 1] and the walk encodes A/s; the CKS schedule of Eq. "fx" takes the
// smallest eigenvalue magnitude of that matrix; Table I, note a).
//
// Two methods, chosen by size:
//   * dimension <= kDenseMax: the dense matrix is reduced to tridiagonal form
//     by Householder reflections (Golub & Van Loan, Sec. 8.3.1; on the lower
//     triangle, the rows shared by a team of host threads in fixed chunks, so
//     that the result does not depend on the thread count) and the
//     eigenvalue of least magnitude is located by bisection on Sturm counts
//     (the number of negative pivots of T - x I is the number of eigenvalues
//     below x; Golub & Van Loan, Sec. 8.4.1).  Exact up to rounding.
//   * larger: Lanczos with full reorthogonalisation (Golub & Van Loan,
//     Sec. 10.1.4).  On A/s first: when its extreme Ritz values show a
//     definite matrix, min |lambda| is the end of the spectrum nearest 0,
//     accepted once its residual bound |beta_k y_k| falls below 1e-9 of it;
//     an indefinite matrix goes through B = (A/s)^2, whose smallest
//     eigenvalue is min |lambda|^2, with the same test.  At most 600 steps,
//     else QW_ENOTSUP: a caller who needs the figure then passes kappa.
// A complex Hermitian X + iY is handled through the real symmetric
// [[X, -Y], [Y, X]], whose spectrum is that of A with every eigenvalue twice.
#include "qw_kappa.h"

#include <sched.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <limits>
#include <map>
#include <string>
#include <thread>
#include <utility>
#include <vector>

namespace qw {
namespace {

constexpr int64_t kDenseMax = 2048;
constexpr int kLanczosMax = 600;
// The dense reduction splits the rows of each trailing block into kChunks
// fixed chunks; from kThreadedMin rows on, a team of host threads shares them.
constexpr int kChunks = 16;
constexpr int64_t kThreadedMin = 256;

// Sparse real symmetric matrix of dimension m as coordinate triplets.
struct Coo {
  int64_t m = 0;
  std::vector<int64_t> r, c;
  std::vector<double> v;
  void add(int64_t i, int64_t j, double x) {
    if (x == 0.0) return;
    r.push_back(i);
    c.push_back(j);
    v.push_back(x);
  }
  void apply(const std::vector<double>& x, std::vector<double>& y) const {
    std::fill(y.begin(), y.end(), 0.0);
    for (size_t t = 0; t < v.size(); ++t) y[size_t(r[t])] += v[t] * x[size_t(c[t])];
  }
};

// Number of eigenvalues below x of the symmetric tridiagonal (d, e), from the
// signs of the pivots of the LDL^T factorisation of T - x I; a zero pivot is
// replaced by -pivmin.
int64_t sturm_below(const std::vector<double>& d, const std::vector<double>& e, double x, double pivmin) {
  int64_t cnt = 0;
  double q = d[0] - x;
  if (std::fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (size_t i = 1; i < d.size(); ++i) {
    q = (d[i] - x) - e[i - 1] * e[i - 1] / q;
    if (std::fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

double tridiag_norm_bound(const std::vector<double>& d, const std::vector<double>& e) {
  double b = 0.0;
  for (size_t i = 0; i < d.size(); ++i) {
    double r = std::fabs(d[i]);
    if (i > 0) r += std::fabs(e[i - 1]);
    if (i + 1 < d.size()) r += std::fabs(e[i]);
    b = std::max(b, r);
  }
  return b;
}

double pivmin_of(const std::vector<double>& e) {
  double emax = 0.0;
  for (double x : e) emax = std::max(emax, x * x);
  return std::numeric_limits<double>::min() * std::max(1.0, emax);
}

// Least |lambda| of the tridiagonal (d, e): the smallest x with an
// eigenvalue in [-x, x), by bisection down to the last bit.
double tridiag_min_abs(const std::vector<double>& d, const std::vector<double>& e) {
  const double pivmin = pivmin_of(e);
  double lo = 0.0, hi = tridiag_norm_bound(d, e) * (1.0 + 1e-15) + pivmin;
  for (int it = 0; it < 2200 && hi - lo > 0.0; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_below(d, e, mid, pivmin) - sturm_below(d, e, -mid, pivmin) >= 1)
      hi = mid;
    else
      lo = mid;
  }
  return hi;
}

// Smallest eigenvalue of the tridiagonal (d, e), by the same bisection.
double tridiag_min(const std::vector<double>& d, const std::vector<double>& e) {
  const double pivmin = pivmin_of(e);
  const double b = tridiag_norm_bound(d, e) * (1.0 + 1e-15) + pivmin;
  double lo = -b, hi = b;
  for (int it = 0; it < 2200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_below(d, e, mid, pivmin) >= 1)
      hi = mid;
    else
      lo = mid;
  }
  return hi;
}

// Threads of the dense reduction: the CPUs this process may run on, at most
// kChunks.
int host_threads() {
  cpu_set_t set;
  CPU_ZERO(&set);
  const int n = sched_getaffinity(0, sizeof(set), &set) == 0 ? CPU_COUNT(&set) : 1;
  return std::max(1, std::min(n, kChunks));
}

// A barrier for the threads of one reduction (they spin, then yield).
class SpinBarrier {
 public:
  explicit SpinBarrier(int n) : n_(n) {}
  void wait() {
    const int g = gen_.load(std::memory_order_acquire);
    if (count_.fetch_add(1, std::memory_order_acq_rel) == n_ - 1) {
      count_.store(0, std::memory_order_relaxed);
      gen_.fetch_add(1, std::memory_order_acq_rel);
      return;
    }
    for (int spin = 0; gen_.load(std::memory_order_acquire) == g; ++spin)
      if (spin > 2048) std::this_thread::yield();
  }

 private:
  const int n_;
  std::atomic<int> count_{0};
  std::atomic<int> gen_{0};
};

// Householder reduction of the dense symmetric a (m x m, row-major; the lower
// triangle is read and overwritten) to the tridiagonal (d, e), as LAPACK's
// unblocked symmetric reduction does it: for column k, the reflector
// H = I - 2 v v^T that zeroes a[k+2.., k], then p = B v over the lower
// triangle of the trailing block B, q = p - (v^T p) v, and the rank-2 update
// B <- B - 2 (v q^T + q v^T) of the lower triangle (Golub & Van Loan,
// Sec. 8.3.1).  The rows of B are split into kChunks fixed chunks of equal
// area; each chunk's part of p is summed on its own and the parts are added in
// chunk order, so the result does not depend on how many threads ran.
void householder_tridiagonal(std::vector<double>& a, int64_t m, std::vector<double>& d, std::vector<double>& e) {
  d.assign(size_t(m), 0.0);
  e.assign(size_t(std::max<int64_t>(m - 1, 0)), 0.0);
  std::vector<double> v(static_cast<size_t>(m)), p(static_cast<size_t>(m)), q(static_cast<size_t>(m));
  std::vector<std::vector<double>> part(kChunks, std::vector<double>(static_cast<size_t>(m)));
  std::vector<char> skip(static_cast<size_t>(m), 0);
  std::vector<double> kpart(kChunks);

  auto bounds = [](int64_t len, int c) {  // rows [bounds(c), bounds(c + 1)) of chunk c: equal areas
    return c >= kChunks ? len : int64_t(std::floor(double(len) * std::sqrt(double(c) / kChunks)));
  };
  // Thread tid of nt (the chunks c = tid, tid + nt, ...); thread 0 also forms
  // the reflectors.
  auto work = [&](int tid, int nt, SpinBarrier& bar) {
    for (int64_t k = 0; k + 2 < m; ++k) {
      const int64_t len = m - k - 1;
      double* const B = &a[size_t((k + 1) * m + k + 1)];  // B[i * m + j], j <= i
      if (tid == 0) {
        double xn = 0.0;
        for (int64_t i = 0; i < len; ++i) {
          v[size_t(i)] = a[size_t((k + 1 + i) * m + k)];
          xn += v[size_t(i)] * v[size_t(i)];
        }
        xn = std::sqrt(xn);
        d[size_t(k)] = a[size_t(k * m + k)];
        skip[size_t(k)] = 1;
        if (xn != 0.0) {
          const double alpha = v[0] > 0.0 ? -xn : xn;
          v[0] -= alpha;
          double vn = 0.0;
          for (int64_t i = 0; i < len; ++i) vn += v[size_t(i)] * v[size_t(i)];
          vn = std::sqrt(vn);
          e[size_t(k)] = alpha;
          if (vn != 0.0) {
            for (int64_t i = 0; i < len; ++i) v[size_t(i)] /= vn;
            skip[size_t(k)] = 0;
          }
        }
      }
      bar.wait();
      if (skip[size_t(k)]) continue;  // thread 0 writes the next column's entry only
      // p = B v from the lower triangle, one partial sum per chunk
      for (int c = tid; c < kChunks; c += nt) {
        const int64_t r0 = bounds(len, c), r1 = bounds(len, c + 1);
        double* pc = part[size_t(c)].data();
        std::fill(pc, pc + r1, 0.0);
        for (int64_t i = r0; i < r1; ++i) {
          const double* row = B + i * m;
          const double vi = v[size_t(i)];
          double t = row[i] * vi;
          for (int64_t j = 0; j < i; ++j) {
            t += row[j] * v[size_t(j)];
            pc[j] += row[j] * vi;
          }
          pc[i] += t;
        }
      }
      bar.wait();
      // p by index slices (the chunks' parts added in chunk order), and v^T p
      for (int c = tid; c < kChunks; c += nt) {
        const int64_t i0 = len * c / kChunks, i1 = len * (c + 1) / kChunks;
        double kp = 0.0;
        for (int64_t i = i0; i < i1; ++i) {
          double t = 0.0;
          for (int h = 0; h < kChunks; ++h)
            if (i < bounds(len, h + 1)) t += part[size_t(h)][size_t(i)];
          p[size_t(i)] = t;
          kp += v[size_t(i)] * t;
        }
        kpart[size_t(c)] = kp;
      }
      bar.wait();
      double K = 0.0;
      for (int c = 0; c < kChunks; ++c) K += kpart[size_t(c)];
      for (int c = tid; c < kChunks; c += nt) {
        const int64_t i0 = len * c / kChunks, i1 = len * (c + 1) / kChunks;
        for (int64_t i = i0; i < i1; ++i) q[size_t(i)] = p[size_t(i)] - K * v[size_t(i)];
      }
      bar.wait();
      // B <- B - 2 (v q^T + q v^T) on the lower triangle
      for (int c = tid; c < kChunks; c += nt) {
        const int64_t r0 = bounds(len, c), r1 = bounds(len, c + 1);
        for (int64_t i = r0; i < r1; ++i) {
          double* row = B + i * m;
          const double vi = 2.0 * v[size_t(i)], qi = 2.0 * q[size_t(i)];
          for (int64_t j = 0; j <= i; ++j) row[j] -= vi * q[size_t(j)] + qi * v[size_t(j)];
        }
      }
      bar.wait();
    }
  };

  int nt = m >= kThreadedMin ? host_threads() : 1;
  std::vector<std::thread> team;
  std::atomic<int> go{0};  // 1: run; 2: not every thread could be started, leave
  SpinBarrier bar(nt);
  if (nt > 1) {
    try {
      team.reserve(size_t(nt - 1));
      for (int t = 1; t < nt; ++t)
        team.emplace_back([&, t] {
          while (go.load(std::memory_order_acquire) == 0) std::this_thread::yield();
          if (go.load(std::memory_order_acquire) == 1) work(t, nt, bar);
        });
      go.store(1, std::memory_order_release);
    } catch (...) {
      go.store(2, std::memory_order_release);
      for (auto& t : team) t.join();
      team.clear();
      nt = 1;
    }
  }
  if (nt > 1) {
    work(0, nt, bar);
  } else {
    SpinBarrier alone(1);
    work(0, 1, alone);
  }
  for (auto& t : team) t.join();
  if (m >= 2) {
    d[size_t(m - 2)] = a[size_t((m - 2) * m + m - 2)];
    e[size_t(m - 2)] = a[size_t((m - 1) * m + m - 2)];
  }
  d[size_t(m - 1)] = a[size_t((m - 1) * m + m - 1)];
}

double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double t = 0.0;
  for (size_t i = 0; i < a.size(); ++i) t += a[i] * b[i];
  return t;
}

// Last component of the eigenvector of the tridiagonal (d, e) for the
// eigenvalue theta (inverse iteration, two sweeps from a flat start).
double tridiag_last_component(const std::vector<double>& d, const std::vector<double>& e, double theta) {
  const size_t k = d.size();
  std::vector<double> x(k, 1.0), y(k), c(k), dd(k);
  const double shift = theta + 1e-14 * std::max(1.0, std::fabs(theta));
  for (int sweep = 0; sweep < 3; ++sweep) {
    // solve (T - shift I) y = x by the Thomas algorithm (no pivoting; the
    // shift is off every eigenvalue by construction of the perturbation)
    dd[0] = d[0] - shift;
    y[0] = x[0];
    for (size_t i = 1; i < k; ++i) {
      const double piv = dd[i - 1] != 0.0 ? dd[i - 1] : 1e-300;
      c[i] = e[i - 1] / piv;
      dd[i] = d[i] - shift - c[i] * e[i - 1];
      y[i] = x[i] - c[i] * y[i - 1];
    }
    y[k - 1] /= dd[k - 1] != 0.0 ? dd[k - 1] : 1e-300;
    for (size_t i = k - 1; i-- > 0;) y[i] = (y[i] - e[i] * y[i + 1]) / (dd[i] != 0.0 ? dd[i] : 1e-300);
    const double n = std::sqrt(dot(y, y));
    for (size_t i = 0; i < k; ++i) x[i] = y[i] / n;
  }
  return x[k - 1];
}

// Lanczos with full reorthogonalisation on A (square = false) or on B = A^2
// (square = true) from a fixed pseudo-random start (64-bit LCG).  Every ten
// steps the extreme Ritz values and their residual bounds are checked:
//   * on A, a converged smallest Ritz value above 0 (largest below 0) is the
//     eigenvalue of least magnitude of a definite matrix: returns it in
//     *out; converged extremes of opposite signs (an indefinite matrix,
//     whose least |lambda| is interior) return 1;
//   * on A^2, the converged smallest Ritz value is min |lambda|^2.
// Converged: residual bound at most 1e-9 of the Ritz value.  Not converged
// after kLanczosMax steps: -5 (QW_ENOTSUP) with the last estimate in *out.
int lanczos(const Coo& A, bool square, double* out, std::string& err) {
  const int64_t m = A.m;
  const int kmax = int(std::min<int64_t>(m, kLanczosMax));
  std::vector<std::vector<double>> V;
  std::vector<double> alpha, beta;
  std::vector<double> v(static_cast<size_t>(m)), w(static_cast<size_t>(m)), t(static_cast<size_t>(m));
  uint64_t st = 0x9e3779b97f4a7c15ull;
  for (int64_t i = 0; i < m; ++i) {
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    v[size_t(i)] = double(int64_t(st >> 11)) / double(int64_t(1) << 53) - 0.5;
  }
  const double nv = std::sqrt(dot(v, v));
  for (double& x : v) x /= nv;
  double est = 0.0;
  for (int k = 0; k < kmax; ++k) {
    V.push_back(v);
    if (square) {
      A.apply(v, t);
      A.apply(t, w);
    } else {
      A.apply(v, w);
    }
    const double a = dot(v, w);
    alpha.push_back(a);
    for (int pass = 0; pass < 2; ++pass)
      for (const auto& q : V) {
        const double h = dot(q, w);
        for (int64_t i = 0; i < m; ++i) w[size_t(i)] -= h * q[size_t(i)];
      }
    const double b = std::sqrt(dot(w, w));
    const bool exhausted = b <= 1e-14 * std::max(1.0, std::fabs(a));  // invariant subspace: Ritz values exact
    const bool last = k + 1 == kmax || exhausted;
    if (k % 10 == 9 || last) {
      const std::vector<double> e(beta.begin(), beta.end());
      const double lo = tridiag_min(alpha, e);
      std::vector<double> na(alpha.size());
      for (size_t i = 0; i < na.size(); ++i) na[i] = -alpha[i];
      const double hi = -tridiag_min(na, e);
      const double rlo = exhausted ? 0.0 : b * std::fabs(tridiag_last_component(alpha, e, lo));
      const double rhi = exhausted ? 0.0 : b * std::fabs(tridiag_last_component(na, e, -hi));
      const bool clo = rlo <= 1e-9 * std::fabs(lo), chi = rhi <= 1e-9 * std::fabs(hi);
      if (square) {
        est = lo;
        if (clo && lo > 0.0) {
          *out = lo;
          return 0;
        }
      } else {
        est = lo > 0.0 ? lo : (hi < 0.0 ? -hi : 0.0);
        if (lo > 0.0 && clo) {
          *out = lo;
          return 0;
        }
        if (hi < 0.0 && chi) {
          *out = -hi;
          return 0;
        }
        if (lo < 0.0 && hi > 0.0 && clo && chi) return 1;  // indefinite
      }
    }
    if (last) break;
    beta.push_back(b);
    for (int64_t i = 0; i < m; ++i) v[size_t(i)] = w[size_t(i)] / b;
  }
  *out = est;
  err = std::string("the Lanczos estimate of min |lambda| (") + (square ? "on (A/s)^2" : "on A/s") +
        ") did not converge in " + std::to_string(kmax) + " steps; pass kappa to the solver";
  return -5;  // QW_ENOTSUP
}

}  // namespace

int min_abs_eigenvalue(int32_t n, int32_t s, int32_t nbits, const int32_t* col, const double* val,
                       const double* vim_home, bool angles, double* lam, std::string& err) {
  // A/s restricted to the n x n matrix the caller gave (padding rows and
  // columns are empty and carry no eigenvalue of the problem).  Row j of the
  // QRAM table holds column j of A: A[col][j] = value.  Fixed-point data
  // holds the rotation angle y of each slot (units of pi); the walk then
  // encodes A'_{col, j} = sign(y) sin^2(pi |y|).
  std::map<std::pair<int64_t, int64_t>, std::pair<double, double>> ent;
  bool cplx = false;
  for (int32_t j = 0; j < n; ++j)
    for (int l = 0; l < s; ++l) {
      const size_t q = size_t(j) * size_t(s) + size_t(l);
      const int32_t c = col[q];
      double re = val[q];
      if (angles) {
        const double sn = std::sin(M_PI * std::fabs(re));
        re = (re < 0.0 ? -1.0 : 1.0) * sn * sn;
        if (val[q] == 0.0) re = 0.0;
      }
      const double im = vim_home ? vim_home[(int64_t(l) << nbits) + j] : 0.0;
      if (re == 0.0 && im == 0.0) continue;
      if (c >= n) {
        err = "a stored entry lies outside the matrix";
        return -1;
      }
      ent[{c, j}] = {re / s, im / s};
      cplx = cplx || im != 0.0;
    }
  for (const auto& kv : ent) {
    const auto it = ent.find({kv.first.second, kv.first.first});
    if (it == ent.end() || it->second.first != kv.second.first || it->second.second != -kv.second.second) {
      err = "kappa is computed for symmetric (Hermitian) matrices only";
      return -5;  // QW_ENOTSUP
    }
  }
  // the real symmetric form: A itself, or [[X, -Y], [Y, X]] for A = X + iY
  Coo A;
  A.m = cplx ? 2 * int64_t(n) : int64_t(n);
  for (const auto& kv : ent) {
    const int64_t r = kv.first.first, c = kv.first.second;
    const double x = kv.second.first, y = kv.second.second;
    A.add(r, c, x);
    if (cplx) {
      A.add(r + n, c + n, x);
      A.add(r, c + n, -y);
      A.add(r + n, c, y);
    }
  }
  double mn;
  if (A.m <= kDenseMax) {
    std::vector<double> a(size_t(A.m) * size_t(A.m), 0.0);
    for (size_t t = 0; t < A.v.size(); ++t) a[size_t(A.r[t] * A.m + A.c[t])] += A.v[t];
    std::vector<double> d, e;
    householder_tridiagonal(a, A.m, d, e);
    mn = tridiag_min_abs(d, e);
  } else {
    // a definite matrix (the solver's usual case) has its least |lambda| at
    // an end of the spectrum, where Lanczos on A converges; an indefinite one
    // goes through (A/s)^2
    double b;
    int rc = lanczos(A, false, &b, err);
    if (rc == 1) {
      rc = lanczos(A, true, &b, err);
      b = std::sqrt(b);
    }
    if (rc) return rc;
    mn = b;
  }
  // below the rounding level of the reduction the matrix is singular as far
  // as double precision can tell (and the schedule would not fit anyway)
  std::vector<double> rowsum(size_t(A.m), 0.0);
  for (size_t t = 0; t < A.v.size(); ++t) rowsum[size_t(A.r[t])] += std::fabs(A.v[t]);
  const double anorm = rowsum.empty() ? 0.0 : *std::max_element(rowsum.begin(), rowsum.end());
  if (!(mn > 64.0 * double(A.m) * std::numeric_limits<double>::epsilon() * anorm)) {
    err = "the matrix is singular to double precision (min |lambda| = " + std::to_string(mn) +
          "): no condition number";
    return -1;
  }
  *lam = mn;
  return 0;
}

}  // namespace qw
