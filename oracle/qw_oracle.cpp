// Quantum-walk oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, single-threaded CPU model of the register-level sparse-state
// simulation of the quantum walk on a sparse Hermitian matrix stored in QRAM
// (Chen et al., "Scalable Program Implementation and Simulation of the
// Large-Scale Quantum Algorithm", arXiv:2303.06890).  Only the test suite, the
// smoke check and the benchmark's CPU-baseline leg may load it; the product
// path never does.  It shares no code with the GPU library.
//
// The state is an ordered map from the full register tuple
// (j_c, j, b1, k_c, k, b2, A) to a complex double (A is the data register:
// one 64-bit word for a real value, two for a complex one), i.e. the "state array +
// amplitude vector" of Sec. V.A ("Main idea") with only nonzero branches kept.
// Every operator is applied literally, one register-level operation at a time:
//   * semi-quantum (per-branch) maps: QRAM/O_A' (XOR of the value word into the
//     A register), O_s' and its inverse (Eq. "Newprocess"), the phase flip P,
//     the swap S;
//   * interference operations (Sec. V.A, "Classical simulation of the
//     interference operation"): group branches whose idle registers agree,
//     apply the small dense matrix to the group (missing members are zero),
//     drop exact zeros.
// T~ follows Alg. 5 step by step, T~^dagger is its exact reverse, and one walk
// step is W = S T~ P T~^dagger (Alg. 6).  Branches with |Re| and |Im| both at or
// below tau are removed at the end of every full W, W^dagger or T~ (never in
// between: inside a step only exact zeros are dropped).
//
// Readings of the paper taken here (each is listed with its reason in the
// design notes of the repository):
//   * P = 2 sum_j |j~><j~| - 1: flip the sign unless b1 = k = b2 = j_c = k_c = 0
//     (Eq. "impl").
//   * The Hadamard acts on the low log2(s) qubits of register k.
//   * R(a, j, k) = [[f, -g], [g, conj f]], f = sqrt(a) for a >= 0,
//     f = +i sqrt|a| if j <= k and -i sqrt|a| if j > k for a < 0,
//     g = sqrt(1 - |a|)  (Sec. IV, footnote on negative elements).  For a
//     complex value off the real axis, f = the principal sqrt(a) (the row of
//     j holds A*_{jk} of a Hermitian matrix, so this is sqrt(A*_{jk}) of
//     psi_j, Sec. IV) and g = sqrt(1 - |a|).
//   * O_s' uses the relative slot index l (Eq. "Newprocess").
//   * Padding: each column gets s sorted unique slots; the filler indices are
//     the smallest row indices missing from that column, with value 0.
//   * s = 2^ceil(log2 max nnz per column) (Table I, note b); N is padded to a
//     power of two with empty columns; register width n = log2 N.
//   * Fixed-point data of word length w (Sec. V.B; appendix table of basic
//     operations): a value is +-q / 2^w with 0 <= q < 2^w; the QRAM word is
//     sign-magnitude; the square-root register holds floor(sqrt(q / 2^w) 2^w)
//     (truncation), the angle register the nearest integer t to
//     arccos(r / 2^w) / (pi/2) * 2^w, and the rotation is by theta =
//     t (pi/2) / 2^w: f = cos(theta) (with the +-i rule for a negative word),
//     g = sin(theta).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <map>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

namespace {

using cplx = std::complex<double>;

// A holds the 64-bit word of a value's real part, A2 that of its imaginary
// part (zero for real matrices): together the data register that O_A' loads.
struct Reg {
  uint64_t jc, j, b1, kc, k, b2, A, A2;
  bool operator<(const Reg& o) const {
    return std::tie(jc, j, b1, kc, k, b2, A, A2) < std::tie(o.jc, o.j, o.b1, o.kc, o.k, o.b2, o.A, o.A2);
  }
  bool operator==(const Reg& o) const {
    return jc == o.jc && j == o.j && b1 == o.b1 && kc == o.kc && k == o.k && b2 == o.b2 && A == o.A &&
           A2 == o.A2;
  }
};

using State = std::map<Reg, cplx>;

struct Matrix {
  int32_t n_orig = 0;
  int32_t N = 0;      // padded dimension (power of two)
  int32_t nbits = 0;  // log2 N
  int32_t s = 0;      // slots per row (power of two)
  int32_t hbits = 0;  // log2 s
  double scale = 1.0;
  std::vector<int32_t> col;   // N*s, row j: sorted unique indices
  std::vector<double> val;    // N*s, real part of the stored value
  std::vector<double> vim;    // N*s, imaginary part (all zero for a real matrix)
  std::vector<uint8_t> real;  // N*s, 1 for a stored entry, 0 for filler
  bool complex_values = false;
  // Fixed-point data (word > 0): slot q's QRAM word is words[q], the sign in
  // bit 63 and the magnitude q' of the value +-q' / 2^word in the low bits.
  int32_t word = 0;
  std::vector<uint64_t> words;
};

std::string g_err;

void fail(const std::string& m) { throw std::runtime_error(m); }

uint64_t bits_of(double v) {
  uint64_t b;
  std::memcpy(&b, &v, 8);
  return b;
}
double double_of(uint64_t b) {
  double v;
  std::memcpy(&v, &b, 8);
  return v;
}

int ceil_log2(int64_t x) {
  int r = 0;
  while ((int64_t(1) << r) < x) ++r;
  return r;
}

// Quantum binary search as a per-branch function (Definition of QBS, Alg. 1):
// left/right/mid/flag, floor midpoint, ceil(log s)+1 fixed iterations; the
// output is the position of `target` in the sorted row, or 0 if it is absent.
uint64_t qbs(const int32_t* row, int s, uint64_t target) {
  int64_t left = 0, right = s;
  bool flag = true;
  uint64_t out = 0;
  const int iters = ceil_log2(s) + 1;
  for (int it = 0; it < iters; ++it) {
    if (!flag) continue;
    const int64_t mid = (left + right) / 2;
    const uint64_t midval = uint64_t(int64_t(row[mid]));
    const bool less = midval < target;
    const bool equal = midval == target;
    if (equal) {
      out ^= uint64_t(mid);
      flag = false;
    } else if (less) {
      left = mid;
    } else {
      right = mid;
    }
  }
  return out;
}

// --- semi-quantum operations ------------------------------------------------

template <class F>
void per_branch(State& st, F f) {
  State out;
  for (auto& kv : st) {
    Reg r = kv.first;
    cplx a = kv.second;
    f(r, a);
    auto ins = out.emplace(r, a);
    if (!ins.second) fail("per-branch map is not injective");
  }
  st.swap(out);
}

// O_A' (Alg. 3): A ^= word(a_{j,l}) where register k holds the slot l (for
// a complex value, both words: real part into A, imaginary part into A2; for
// fixed-point data, the sign-magnitude fixed-point word).
void op_OA(State& st, const Matrix& m) {
  per_branch(st, [&](Reg& r, cplx&) {
    if (r.k >= uint64_t(m.s) || r.j >= uint64_t(m.N)) fail("O_A' address outside the row");
    if (m.word > 0) {
      r.A ^= m.words[r.j * m.s + r.k];
      return;
    }
    r.A ^= bits_of(m.val[r.j * m.s + r.k]);
    r.A2 ^= bits_of(m.vim[r.j * m.s + r.k]);
  });
}

// O_s' (Eq. Newprocess): |j>|l>|z> -> |j>|z ^ k_{j,l}>|l ^ i_j(z ^ k_{j,l})>,
// with l in register k and z in register k_c.
void op_OS(State& st, const Matrix& m) {
  per_branch(st, [&](Reg& r, cplx&) {
    const uint64_t l = r.k, z = r.kc;
    if (l >= uint64_t(m.s)) fail("O_s' slot index >= s");
    const int32_t* row = &m.col[r.j * m.s];
    const uint64_t k = z ^ uint64_t(row[l]);
    const uint64_t kc = l ^ qbs(row, m.s, k);
    r.k = k;
    r.kc = kc;
  });
}

// Inverse of O_s': l = k_c ^ i_j(k), z = k ^ k_{j,l}.
void op_OSinv(State& st, const Matrix& m) {
  per_branch(st, [&](Reg& r, cplx&) {
    const uint64_t k = r.k, kc = r.kc;
    const int32_t* row = &m.col[r.j * m.s];
    const uint64_t l = kc ^ qbs(row, m.s, k);
    if (l >= uint64_t(m.s)) fail("O_s'^-1 produced a slot index >= s");
    const uint64_t z = k ^ uint64_t(row[l]);
    r.k = l;
    r.kc = z;
  });
}

// P = 2 sum_j |j~><j~| - 1.
void op_P(State& st) {
  for (auto& kv : st) {
    const Reg& r = kv.first;
    if (r.A != 0 || r.A2 != 0) fail("A register not clean at P");
    const bool zero = r.jc == 0 && r.b1 == 0 && r.kc == 0 && r.k == 0 && r.b2 == 0;
    if (!zero) kv.second = -kv.second;
  }
}

// S: (j_c, j, b1) <-> (k_c, k, b2).
void op_S(State& st) {
  per_branch(st, [&](Reg& r, cplx&) {
    std::swap(r.jc, r.kc);
    std::swap(r.j, r.k);
    std::swap(r.b1, r.b2);
  });
}

// --- interference operations -------------------------------------------------

// H^{(x) log2 s} on the low log2(s) qubits of register k.  Groups: all
// registers equal except those qubits.
void op_H(State& st, const Matrix& m) {
  const uint64_t mask = uint64_t(m.s) - 1;
  std::map<Reg, std::vector<cplx>> groups;
  for (auto& kv : st) {
    Reg g = kv.first;
    const uint64_t x = g.k & mask;
    g.k &= ~mask;
    auto& v = groups[g];
    if (v.empty()) v.assign(m.s, cplx(0.0, 0.0));
    v[x] = kv.second;
  }
  const double inv = 1.0 / std::sqrt(double(m.s));
  State out;
  for (auto& gv : groups) {
    const std::vector<cplx>& v = gv.second;
    for (int x = 0; x < m.s; ++x) {
      cplx acc(0.0, 0.0);
      for (int y = 0; y < m.s; ++y) {
        if (__builtin_popcount(unsigned(x & y)) & 1)
          acc -= v[y];
        else
          acc += v[y];
      }
      acc *= inv;
      if (acc.real() != 0.0 || acc.imag() != 0.0) {
        Reg r = gv.first;
        r.k |= uint64_t(x);
        out.emplace(r, acc);
      }
    }
  }
  st.swap(out);
}

struct Rot {
  cplx f;
  double g;
};

// Amplitudes of the conditional rotation on b2 for the value a + i b held in
// row j at column k: f = sqrt(a + i b) (the principal root; the row holds
// A*_{jk} of a Hermitian matrix, so this is the sqrt(A*_{jk}) of psi_j), with
// the footnote's rule on the negative real axis, where the principal root is
// not conjugation-symmetric: f = +i sqrt|a| when j <= k, -i sqrt|a| otherwise;
// g = sqrt(1 - |a + i b|).
Rot rotation(double a, double b, uint64_t j, uint64_t k) {
  Rot r;
  if (b != 0.0) {
    r.f = std::sqrt(cplx(a, b));
    r.g = std::sqrt(1.0 - std::abs(cplx(a, b)));
    return r;
  }
  if (a >= 0.0) {
    r.f = cplx(std::sqrt(a), 0.0);
  } else {
    const double q = std::sqrt(-a);
    r.f = (j <= k) ? cplx(0.0, q) : cplx(0.0, -q);
  }
  r.g = std::sqrt(1.0 - std::fabs(a));
  return r;
}

// Derivatives df/da, dg/da of the rotation amplitudes (not finite at a = 0 and
// at |a| = 1).
Rot rotation_deriv(double a, uint64_t j, uint64_t k) {
  Rot d;
  if (a > 0.0) {
    d.f = cplx(0.5 / std::sqrt(a), 0.0);
  } else if (a < 0.0) {
    const double q = -0.5 / std::sqrt(-a);
    d.f = (j <= k) ? cplx(0.0, q) : cplx(0.0, -q);
  } else {
    d.f = cplx(INFINITY, 0.0);
  }
  const double sg = a > 0.0 ? 1.0 : (a < 0.0 ? -1.0 : 0.0);
  d.g = -sg * 0.5 / std::sqrt(1.0 - std::fabs(a));
  return d;
}

// ---- fixed-point rotation (Sec. V.B: values are fixed-point numbers of a
// given word length; appendix table of basic operations: the conditional
// rotation is computed with a fixed-point square root, a fixed-point arccos
// and a rotation by a fixed-point angle) --------------------------------------

// floor(sqrt(x)) for any 64-bit x.
uint64_t isqrt64(uint64_t x) {
  uint64_t r = uint64_t(std::sqrt((long double)x));
  while (r > 0 && (unsigned __int128)r * r > x) --r;
  while ((unsigned __int128)(r + 1) * (r + 1) <= x) ++r;
  return r;
}

// The square-root register: sqrt(q / 2^w) truncated to w fraction bits, as an
// integer in [0, 2^w).
uint64_t fx_sqrt(uint64_t q, int w) { return isqrt64(q << w); }

// The angle register: arccos of the fixed-point r / 2^w in units of
// (pi/2) / 2^w, rounded to the nearest integer (0 ... 2^w).
uint64_t fx_arccos(uint64_t r, int w) {
  const double x = double(r) / double(uint64_t(1) << w);
  return uint64_t(std::nearbyint(std::acos(x) * (double(uint64_t(1) << (w + 1)) / M_PI)));
}

// cos and sin of the angle t (pi/2) / 2^w, exact at 0 and pi/2 and taken
// from the nearer end of the quarter turn otherwise.
void quarter_cos_sin(uint64_t t, int w, double& c, double& sn) {
  const uint64_t full = uint64_t(1) << w;
  const auto ang = [&](uint64_t u) { return (M_PI / 2.0) * (double(u) / double(full)); };
  c = t == full ? 0.0 : (2 * t <= full ? std::cos(ang(t)) : std::sin(ang(full - t)));
  sn = t == 0 ? 0.0 : (2 * t >= full ? std::cos(ang(full - t)) : std::sin(ang(t)));
}

// Rotation amplitudes for the fixed-point word A (sign bit 63, magnitude in
// the low w bits) held by row j at column k: theta = the angle register, f =
// cos(theta) (times +-i for a negative word, by the rule of the real case),
// g = sin(theta).
Rot rotation_fixed(uint64_t A, int w, uint64_t j, uint64_t k) {
  const uint64_t q = A & ((uint64_t(1) << w) - 1);
  const bool neg = (A >> 63) != 0;
  double c, sn;
  quarter_cos_sin(fx_arccos(fx_sqrt(q, w), w), w, c, sn);
  Rot r;
  r.f = !neg ? cplx(c, 0.0) : ((j <= k) ? cplx(0.0, c) : cplx(0.0, -c));
  r.g = sn;
  return r;
}

// 2x2 matrix [[m00, m01], [m10, m11]] of R (dagger=false) or R^dagger.
void rot_matrix(const Rot& r, bool dagger, cplx M[2][2]) {
  if (!dagger) {
    M[0][0] = r.f;
    M[0][1] = -r.g;
    M[1][0] = r.g;
    M[1][1] = std::conj(r.f);
  } else {
    M[0][0] = std::conj(r.f);
    M[0][1] = r.g;
    M[1][0] = -r.g;
    M[1][1] = r.f;
  }
}

// Conditional rotation on b2 controlled by the A register (value), j and k.
void op_CR(State& st, const Matrix& m, bool dagger) {
  std::map<Reg, std::pair<cplx, cplx>> groups;
  for (auto& kv : st) {
    Reg g = kv.first;
    const uint64_t b = g.b2;
    g.b2 = 0;
    auto& p = groups[g];
    (b ? p.second : p.first) = kv.second;
  }
  State out;
  for (auto& gv : groups) {
    const Reg& g = gv.first;
    const Rot r = m.word > 0 ? rotation_fixed(g.A, m.word, g.j, g.k)
                             : rotation(double_of(g.A), double_of(g.A2), g.j, g.k);
    cplx M[2][2];
    rot_matrix(r, dagger, M);
    const cplx v0 = gv.second.first, v1 = gv.second.second;
    const cplx o0 = M[0][0] * v0 + M[0][1] * v1;
    const cplx o1 = M[1][0] * v0 + M[1][1] * v1;
    if (o0.real() != 0.0 || o0.imag() != 0.0) {
      Reg q = g;
      q.b2 = 0;
      out.emplace(q, o0);
    }
    if (o1.real() != 0.0 || o1.imag() != 0.0) {
      Reg q = g;
      q.b2 = 1;
      out.emplace(q, o1);
    }
  }
  st.swap(out);
}

// --- the walk as a list of register-level operations --------------------------

enum Op { H, OA, OS, OSINV, CR, CRDAG, P, S };

// T~ (Alg. 5): Hadamard on k; O_A'; O_s'; rotation; O_s'^dagger; O_A'
// (uncompute); O_s'.
const std::vector<Op> kT = {H, OA, OS, CR, OSINV, OA, OS};
// T~^dagger: the same list reversed, each operation inverted.
const std::vector<Op> kTdag = {OSINV, OA, OS, CRDAG, OSINV, OA, H};

std::vector<Op> walk_ops() {
  std::vector<Op> w = kTdag;
  w.push_back(P);
  w.insert(w.end(), kT.begin(), kT.end());
  w.push_back(S);
  return w;
}

// W^dagger = T~ P T~^dagger S applied as S first, then T~^dagger, P, T~.
std::vector<Op> walk_dag_ops() {
  std::vector<Op> w = {S};
  w.insert(w.end(), kTdag.begin(), kTdag.end());
  w.push_back(P);
  w.insert(w.end(), kT.begin(), kT.end());
  return w;
}

Op inverse(Op o) {
  switch (o) {
    case OS: return OSINV;
    case OSINV: return OS;
    case CR: return CRDAG;
    case CRDAG: return CR;
    default: return o;
  }
}

void apply(State& st, const Matrix& m, Op o) {
  switch (o) {
    case H: op_H(st, m); break;
    case OA: op_OA(st, m); break;
    case OS: op_OS(st, m); break;
    case OSINV: op_OSinv(st, m); break;
    case CR: op_CR(st, m, false); break;
    case CRDAG: op_CR(st, m, true); break;
    case P: op_P(st); break;
    case S: op_S(st); break;
  }
}

struct OState {
  const Matrix* m;
  State st;
  double tau = 1e-13;
  double margin = 1e-15;
  int64_t ambiguous = 0;       // amplitudes within +-margin of tau at the last prune
  int64_t ambiguous_total = 0;  // summed over all prunes
  double pruned_mass = 0.0;     // sum |amp|^2 removed by the last prune
  int64_t max_size = 0;         // largest number of branches after any single operation
};

void prune(OState& o) {
  int64_t amb = 0;
  double mass = 0.0;
  for (auto it = o.st.begin(); it != o.st.end();) {
    const double mx = std::max(std::fabs(it->second.real()), std::fabs(it->second.imag()));
    if (std::fabs(mx - o.tau) <= o.margin) ++amb;
    if (mx <= o.tau) {
      mass += std::norm(it->second);
      it = o.st.erase(it);
    } else {
      ++it;
    }
  }
  o.ambiguous = amb;
  o.ambiguous_total += amb;
  o.pruned_mass = mass;
}

// Apply the operations in order, keeping the largest intermediate size (the
// M_max of the space-complexity discussion, Sec. "The space complexity of
// simulating the quantum walk", counts the branches inside a step).
void run(OState& o, const std::vector<Op>& ops) {
  for (Op op : ops) {
    apply(o.st, *o.m, op);
    o.max_size = std::max<int64_t>(o.max_size, int64_t(o.st.size()));
  }
}

uint64_t pack(const Matrix& m, const Reg& r) {
  const int n = m.nbits;
  uint64_t key = r.jc;
  key = (key << n) | r.j;
  key = (key << 1) | r.b1;
  key = (key << n) | r.kc;
  key = (key << n) | r.k;
  key = (key << 1) | r.b2;
  return key;
}

Reg unpack(const Matrix& m, uint64_t key) {
  const int n = m.nbits;
  const uint64_t nm = (uint64_t(1) << n) - 1;
  Reg r{};
  r.b2 = key & 1;
  key >>= 1;
  r.k = key & nm;
  key >>= n;
  r.kc = key & nm;
  key >>= n;
  r.b1 = key & 1;
  key >>= 1;
  r.j = key & nm;
  key >>= n;
  r.jc = key & nm;
  r.A = 0;
  r.A2 = 0;
  return r;
}

template <class F>
int guarded(F f) {
  try {
    f();
    return 0;
  } catch (const std::exception& e) {
    g_err = e.what();
    return -1;
  }
}

// ---- Chebyshev-series coefficients (Eq. "fx") ---------------------------------
// a_j = 4 (-1)^j sum_{i=j+1}^{beta} C(2 beta, beta+i) / 2^{2 beta}, computed
// from log-gamma in long double and summed from the far tail inwards.
void cks_coeffs(int64_t beta, int32_t j0, double* out) {
  const long double ln2 = std::log(2.0L);
  const long double lg2b = std::lgamma((long double)(2 * beta + 1));
  // terms beyond 60 standard deviations are far below double precision
  const long double sd = std::sqrt((long double)beta / 2.0L);
  int64_t imax = std::min<int64_t>(beta, int64_t(j0) + 2 + int64_t(60.0L * sd + 10.0L));
  std::vector<long double> suffix(imax + 2, 0.0L);
  for (int64_t i = imax; i >= 0; --i) {
    const long double lp = lg2b - std::lgamma((long double)(beta + i + 1)) -
                           std::lgamma((long double)(beta - i + 1)) - 2.0L * beta * ln2;
    suffix[i] = suffix[i + 1] + std::exp(lp);
  }
  for (int32_t j = 0; j <= j0; ++j) {
    const long double tail = (j + 1 <= imax) ? suffix[j + 1] : 0.0L;
    out[j] = double(4.0L * ((j & 1) ? -1.0L : 1.0L) * tail);
  }
}

}  // namespace

// =============================== C interface ==================================
extern "C" {

const char* orc_last_error() { return g_err.c_str(); }

// Preprocessing (Sec. V.B, numbered list): rescale, CSC rows per column, s,
// zero fill.  scale_in > 0 fixes the scale; otherwise 1/max(1, max|a|).
// vals_im: imaginary parts (NULL for a real matrix).  The matrix is taken as
// given (Hermitian or symmetric input is the caller's business).
void* orc_matrix_new(int32_t n, const int32_t* colptr, const int32_t* rowidx, const double* vals,
                     const double* vals_im, int64_t nnz, double scale_in) {
  Matrix* m = new Matrix;
  int rc = guarded([&] {
    if (n <= 0) fail("n must be positive");
    if (colptr[0] != 0 || colptr[n] != nnz) fail("bad colptr");
    double amax = 0.0;
    int64_t smax = 1;
    for (int32_t c = 0; c < n; ++c) {
      if (colptr[c + 1] < colptr[c]) fail("colptr not monotone");
      smax = std::max<int64_t>(smax, colptr[c + 1] - colptr[c]);
      for (int64_t p = colptr[c]; p < colptr[c + 1]; ++p) {
        if (rowidx[p] < 0 || rowidx[p] >= n) fail("row index out of range");
        if (p > colptr[c] && rowidx[p] <= rowidx[p - 1]) fail("row indices not sorted/unique");
        amax = std::max(amax, vals_im ? std::abs(cplx(vals[p], vals_im[p])) : std::fabs(vals[p]));
      }
    }
    m->n_orig = n;
    m->scale = scale_in > 0.0 ? scale_in : 1.0 / std::max(1.0, amax);
    m->nbits = std::max(1, ceil_log2(n));
    m->N = 1 << m->nbits;
    m->hbits = ceil_log2(smax);
    m->s = 1 << m->hbits;
    if (m->s > m->N) fail("s exceeds N");
    m->complex_values = vals_im != nullptr;
    m->col.assign(size_t(m->N) * m->s, 0);
    m->val.assign(size_t(m->N) * m->s, 0.0);
    m->vim.assign(size_t(m->N) * m->s, 0.0);
    m->real.assign(size_t(m->N) * m->s, 0);
    for (int32_t c = 0; c < m->N; ++c) {
      std::vector<std::pair<int32_t, cplx>> ent;
      std::vector<uint8_t> present(m->N, 0);
      if (c < n) {
        for (int64_t p = colptr[c]; p < colptr[c + 1]; ++p) {
          ent.push_back({rowidx[p], cplx(vals[p] * m->scale, vals_im ? vals_im[p] * m->scale : 0.0)});
          present[rowidx[p]] = 1;
        }
      }
      const size_t nreal = ent.size();
      for (int32_t r = 0; int64_t(ent.size()) < m->s; ++r)
        if (!present[r]) ent.push_back({r, cplx(0.0, 0.0)});
      std::vector<uint8_t> isreal(ent.size(), 0);
      for (size_t q = 0; q < nreal; ++q) isreal[q] = 1;
      std::vector<size_t> idx(ent.size());
      for (size_t q = 0; q < idx.size(); ++q) idx[q] = q;
      std::sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return ent[a].first < ent[b].first; });
      for (int l = 0; l < m->s; ++l) {
        m->col[size_t(c) * m->s + l] = ent[idx[l]].first;
        m->val[size_t(c) * m->s + l] = ent[idx[l]].second.real();
        m->vim[size_t(c) * m->s + l] = ent[idx[l]].second.imag();
        m->real[size_t(c) * m->s + l] = isreal[idx[l]];
      }
    }
    for (size_t q = 0; q < m->val.size(); ++q)
      if (std::abs(cplx(m->val[q], m->vim[q])) > 1.0) fail("|a| > 1 after scaling");
  });
  if (rc) {
    delete m;
    return nullptr;
  }
  return m;
}

// Switch a real matrix to fixed-point data of word length w (1 ... 32): every
// scaled value must be +-q / 2^w with an integer 0 <= q < 2^w (the paper's
// elements are fixed-point numbers below 1 in magnitude); its QRAM word is
// the sign in bit 63 and q in the low w bits.
int orc_matrix_set_word(void* p, int32_t w) {
  Matrix* m = static_cast<Matrix*>(p);
  return guarded([&] {
    if (w < 1 || w > 32) fail("word length must be 1 ... 32");
    if (m->complex_values) fail("fixed-point data is defined for real matrices only");
    const double full = double(uint64_t(1) << w);
    std::vector<uint64_t> words(m->val.size(), 0);
    for (size_t q = 0; q < m->val.size(); ++q) {
      const double x = std::fabs(m->val[q]) * full;  // exact: a power-of-two scaling
      if (x != std::floor(x) || x >= full) fail("value is not a fixed-point number of the word length");
      words[q] = uint64_t(x) | (std::signbit(m->val[q]) && x != 0.0 ? uint64_t(1) << 63 : 0);
    }
    m->word = w;
    m->words.swap(words);
  });
}

void orc_matrix_free(void* p) { delete static_cast<Matrix*>(p); }

void orc_matrix_info(void* p, int32_t* N, int32_t* s, int32_t* nbits, double* scale) {
  const Matrix* m = static_cast<Matrix*>(p);
  *N = m->N;
  *s = m->s;
  *nbits = m->nbits;
  *scale = m->scale;
}

void orc_matrix_ell(void* p, int32_t* col, double* val, double* vim, uint8_t* real) {
  const Matrix* m = static_cast<Matrix*>(p);
  std::copy(m->col.begin(), m->col.end(), col);
  std::copy(m->val.begin(), m->val.end(), val);
  std::copy(m->vim.begin(), m->vim.end(), vim);
  std::copy(m->real.begin(), m->real.end(), real);
}

uint64_t orc_qbs(const int32_t* row, int32_t s, uint64_t target) { return qbs(row, s, target); }

// The fixed-point registers and rotation amplitudes, for unit tests.
uint64_t orc_fx_sqrt(uint64_t q, int32_t w) { return fx_sqrt(q, w); }
uint64_t orc_fx_arccos(uint64_t r, int32_t w) { return fx_arccos(r, w); }
void orc_fx_rotation(uint64_t A, int32_t w, uint64_t j, uint64_t k, double* fre, double* fim, double* g) {
  const Rot r = rotation_fixed(A, w, j, k);
  *fre = r.f.real();
  *fim = r.f.imag();
  *g = r.g;
}

void* orc_state_new(void* mat, double tau) {
  OState* o = new OState;
  o->m = static_cast<Matrix*>(mat);
  o->tau = tau;
  return o;
}

void orc_state_free(void* p) { delete static_cast<OState*>(p); }

void* orc_state_clone(void* p) { return new OState(*static_cast<OState*>(p)); }

// |b~> = sum_j b_j |0, j, 0, 0, 0, 0>.
int orc_set_b(void* p, const double* bre, const double* bim, int32_t nb) {
  OState* o = static_cast<OState*>(p);
  return guarded([&] {
    if (nb > o->m->N) fail("b longer than N");
    o->st.clear();
    for (int32_t j = 0; j < nb; ++j) {
      const cplx a(bre[j], bim ? bim[j] : 0.0);
      if (a.real() != 0.0 || a.imag() != 0.0) o->st.emplace(Reg{0, uint64_t(j), 0, 0, 0, 0, 0}, a);
    }
  });
}

int orc_import(void* p, const uint64_t* keys, const double* re, const double* im, int64_t m) {
  OState* o = static_cast<OState*>(p);
  return guarded([&] {
    o->st.clear();
    for (int64_t i = 0; i < m; ++i) {
      const cplx a(re[i], im[i]);
      auto ins = o->st.emplace(unpack(*o->m, keys[i]), a);
      if (!ins.second) ins.first->second += a;
    }
  });
}

// Single operations, for unit tests.  code: 0 H, 1 O_A', 2 O_s', 3 O_s'^-1,
// 4 R, 5 R^dagger, 6 P, 7 S.
int orc_apply_op(void* p, int32_t code) {
  OState* o = static_cast<OState*>(p);
  return guarded([&] { apply(o->st, *o->m, Op(code)); });
}

int orc_apply_T(void* p, int32_t dagger) {
  OState* o = static_cast<OState*>(p);
  return guarded([&] {
    run(*o, dagger ? kTdag : kT);
    prune(*o);
  });
}

int orc_step(void* p, int32_t nsteps) {
  OState* o = static_cast<OState*>(p);
  const std::vector<Op> w = walk_ops();
  return guarded([&] {
    for (int32_t t = 0; t < nsteps; ++t) {
      run(*o, w);
      prune(*o);
    }
  });
}

int orc_step_adjoint(void* p, int32_t nsteps) {
  OState* o = static_cast<OState*>(p);
  const std::vector<Op> w = walk_dag_ops();
  return guarded([&] {
    for (int32_t t = 0; t < nsteps; ++t) {
      run(*o, w);
      prune(*o);
    }
  });
}

int64_t orc_count(void* p) { return int64_t(static_cast<OState*>(p)->st.size()); }

int64_t orc_ambiguous(void* p, int32_t total) {
  const OState* o = static_cast<OState*>(p);
  return total ? o->ambiguous_total : o->ambiguous;
}

double orc_pruned_mass(void* p) { return static_cast<OState*>(p)->pruned_mass; }

// Largest branch count after any single operation so far (inside steps too).
int64_t orc_max_size(void* p) { return static_cast<OState*>(p)->max_size; }

// Export sorted by packed key; fails if an ancilla (A) is not clean.
int orc_export(void* p, uint64_t* keys, double* re, double* im) {
  OState* o = static_cast<OState*>(p);
  return guarded([&] {
    std::vector<std::pair<uint64_t, cplx>> v;
    v.reserve(o->st.size());
    for (auto& kv : o->st) {
      if (kv.first.A != 0 || kv.first.A2 != 0) fail("A register not clean");
      v.push_back({pack(*o->m, kv.first), kv.second});
    }
    std::sort(v.begin(), v.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    for (size_t i = 0; i < v.size(); ++i) {
      keys[i] = v[i].first;
      re[i] = v[i].second.real();
      im[i] = v[i].second.imag();
    }
  });
}

double orc_norm2(void* p) {
  double acc = 0.0;
  for (auto& kv : static_cast<OState*>(p)->st) acc += std::norm(kv.second);
  return acc;
}

// Marginal probability of the j register.
void orc_j_marginal(void* p, double* out) {
  OState* o = static_cast<OState*>(p);
  std::fill(out, out + o->m->N, 0.0);
  for (auto& kv : o->st) out[kv.first.j] += std::norm(kv.second);
}

// y_j = <j~| T~^dagger |state>: apply T~^dagger to a copy and read the
// amplitudes of |0, j, 0, 0, 0, 0>.
int orc_project0(void* p, double* yre, double* yim) {
  OState* o = static_cast<OState*>(p);
  return guarded([&] {
    State st = o->st;
    for (Op op : kTdag) apply(st, *o->m, op);
    std::fill(yre, yre + o->m->N, 0.0);
    std::fill(yim, yim + o->m->N, 0.0);
    for (auto& kv : st) {
      const Reg& r = kv.first;
      if (r.jc == 0 && r.b1 == 0 && r.kc == 0 && r.k == 0 && r.b2 == 0 && r.A == 0 && r.A2 == 0) {
        yre[r.j] = kv.second.real();
        yim[r.j] = kv.second.imag();
      }
    }
  });
}

// ---- linear solver (Eq. "fx", Sec. V.B) --------------------------------------

// beta = ceil(kappa^2 ln(kappa/eps)), j0 = ceil(sqrt(beta ln(4 beta/eps))).
void orc_schedule(double kappa, double eps, int64_t* beta, int32_t* j0) {
  const double b = std::ceil(kappa * kappa * std::log(kappa / eps));
  *beta = int64_t(b);
  *j0 = int32_t(std::ceil(std::sqrt(b * std::log(4.0 * b / eps))));
}

void orc_cks_coeffs(int64_t beta, int32_t j0, double* out) { cks_coeffs(beta, j0, out); }

// Classical truncated series y = sum_{k<=j0} a_k T_{2k+1}(A/s) b by the
// three-term Chebyshev recurrence on the padded, scaled matrix.  Row j of the
// table holds column j of A (entries A_{col, j}), so A x is a scatter:
// (A x)_{col[j,l]} += a_{j,l} x_j.
int orc_cheb_series(void* mat, const double* bre, const double* bim, int32_t nb, int32_t j0,
                    const double* coef, double* yre, double* yim) {
  const Matrix& m = *static_cast<Matrix*>(mat);
  if (m.word > 0) {
    g_err = "the classical series uses the values themselves, not fixed-point data";
    return -1;
  }
  const int N = m.N;
  auto apply_h = [&](const std::vector<cplx>& x, std::vector<cplx>& out) {
    std::fill(out.begin(), out.end(), cplx(0.0, 0.0));
    for (int r = 0; r < N; ++r)
      for (int l = 0; l < m.s; ++l) {
        const size_t q = size_t(r) * m.s + l;
        out[m.col[q]] += cplx(m.val[q], m.vim[q]) * x[r];
      }
    for (int r = 0; r < N; ++r) out[r] /= double(m.s);
  };
  std::vector<cplx> tprev(N, cplx(0.0, 0.0)), tcur(N), tnext(N), hx(N), y(N, cplx(0.0, 0.0));
  for (int r = 0; r < nb; ++r) tprev[r] = cplx(bre[r], bim ? bim[r] : 0.0);  // T_0 b
  apply_h(tprev, tcur);                                                         // T_1 b
  for (int32_t k = 0; k <= j0; ++k) {
    // tcur holds T_{2k+1} b
    for (int r = 0; r < N; ++r) y[r] += coef[k] * tcur[r];
    if (k == j0) break;
    for (int rep = 0; rep < 2; ++rep) {
      apply_h(tcur, hx);
      for (int r = 0; r < N; ++r) tnext[r] = 2.0 * hx[r] - tprev[r];
      tprev.swap(tcur);
      tcur.swap(tnext);
    }
  }
  for (int r = 0; r < N; ++r) {
    yre[r] = y[r].real();
    yim[r] = y[r].imag();
  }
  return 0;
}

// Walk-based solver: omega = W T~ |b~>; for k = 0..j0: y += a_k Pi_0 T~^dagger
// omega; omega = W^2 omega.  y is the unnormalised LCU output (N-vector).
int orc_qls_walk(void* mat, const double* b, int32_t nb, int32_t j0, const double* coef,
                 double tau, double* yre, double* yim) {
  const Matrix& m = *static_cast<Matrix*>(mat);
  OState o;
  o.m = &m;
  o.tau = tau;
  std::vector<double> pr(m.N), pi(m.N);
  return guarded([&] {
    for (int32_t j = 0; j < nb; ++j)
      if (b[j] != 0.0) o.st.emplace(Reg{0, uint64_t(j), 0, 0, 0, 0, 0}, cplx(b[j], 0.0));
    run(o, kT);
    prune(o);
    const std::vector<Op> w = walk_ops();
    run(o, w);
    prune(o);
    std::fill(yre, yre + m.N, 0.0);
    std::fill(yim, yim + m.N, 0.0);
    for (int32_t k = 0; k <= j0; ++k) {
      if (orc_project0(&o, pr.data(), pi.data())) fail(g_err);
      for (int r = 0; r < m.N; ++r) {
        yre[r] += coef[k] * pr[r];
        yim[r] += coef[k] * pi[r];
      }
      if (k == j0) break;
      for (int rep = 0; rep < 2; ++rep) {
        run(o, w);
        prune(o);
      }
    }
  });
}

// d f / d Re v and d g / d Re v (im = false), or the same with respect to
// Im v (im = true), for a complex value v = a + i b.  Off the real axis f is
// the principal sqrt(v), holomorphic there, so df/da = 1/(2f) and
// df/db = i/(2f); g = sqrt(1 - |v|) with d|v|/da = a/|v| and d|v|/db = b/|v|.
// On the axis the real rule of rotation() holds: with respect to a it is
// rotation_deriv; with respect to b the principal root is analytic only for
// a > 0 (df/db = i/(2 sqrt a), dg/db = 0), and for a <= 0 the derivative does
// not exist (NaN: the real rule's +-i branch is one side of the cut).
Rot rotation_deriv_c(double a, double b, uint64_t j, uint64_t k, bool im) {
  if (b == 0.0 && !im) return rotation_deriv(a, j, k);
  Rot d;
  if (b == 0.0) {
    if (a > 0.0) {
      d.f = cplx(0.0, 0.5 / std::sqrt(a));
      d.g = 0.0;
    } else {
      d.f = cplx(NAN, NAN);
      d.g = NAN;
    }
    return d;
  }
  const cplx f = std::sqrt(cplx(a, b));
  const double mod = std::abs(cplx(a, b));
  d.f = (im ? cplx(0.0, 1.0) : cplx(1.0, 0.0)) / (2.0 * f);
  d.g = -(im ? b : a) / (2.0 * mod * std::sqrt(1.0 - mod));
  return d;
}

// ---- reverse-mode gradient with stored states ---------------------------------
// Loss L = sum_j w_j p_j(psi_n), psi_n = W^n T~ |b~>.  Forward: every operation
// of T~ and of the n walk steps is applied in order, and the input state of
// every rotation site (R in T~, R^dagger in T~^dagger) is stored.  Backward:
// lambda = O psi_n with O = diag(w_j) on register j; walking the operations in
// reverse, a rotation site adds 2 Re <lambda_out | dU/da | x_in> to the value
// the site's A register holds (slot l = k_c ^ i_j(k) of row j), and lambda is
// mapped through the inverse operation.  At the start, dL/db_j = 2 lambda(j~).
// dv is indexed by ELL slot (j*s + l).  For a complex matrix dv holds
// dL/dRe v and dvi dL/dIm v, each entry taken as an independent parameter
// (the Hermitian mirror of an entry has its own derivative).
static int grad_impl(void* mat, const double* bre, const double* bim, int32_t nb, int32_t nsteps,
                     const double* w, double tau, double* dv, double* dvi, double* dbre, double* dbim, double* loss) {
  const Matrix& m = *static_cast<Matrix*>(mat);
  return guarded([&] {
    if (m.complex_values && !dvi) fail("a complex matrix takes the complex gradient (orc_grad_complex)");
    if (!m.complex_values && dvi) fail("a real matrix takes orc_grad");
    if (m.word > 0) fail("the gradient is defined for real-valued (not fixed-point) data only");
    OState o;
    o.m = &m;
    o.tau = tau;
    for (int32_t j = 0; j < nb; ++j) {
      const cplx a(bre[j], bim ? bim[j] : 0.0);
      if (a.real() != 0.0 || a.imag() != 0.0) o.st.emplace(Reg{0, uint64_t(j), 0, 0, 0, 0, 0}, a);
    }
    std::vector<Op> prog(kT.begin(), kT.end());
    std::vector<int> prune_after;  // op indices after which the forward pass pruned
    prune_after.push_back(int(prog.size()) - 1);
    const std::vector<Op> wops = walk_ops();
    for (int32_t t = 0; t < nsteps; ++t) {
      prog.insert(prog.end(), wops.begin(), wops.end());
      prune_after.push_back(int(prog.size()) - 1);
    }
    std::vector<State> stored(prog.size());
    size_t pi = 0;
    for (size_t i = 0; i < prog.size(); ++i) {
      if (prog[i] == CR || prog[i] == CRDAG) stored[i] = o.st;
      apply(o.st, m, prog[i]);
      if (pi < prune_after.size() && prune_after[pi] == int(i)) {
        prune(o);
        ++pi;
      }
    }
    double L = 0.0;
    State lam;
    for (auto& kv : o.st) {
      const double wj = w[kv.first.j];
      L += wj * std::norm(kv.second);
      if (wj != 0.0) lam.emplace(kv.first, wj * kv.second);
    }
    *loss = L;
    std::fill(dv, dv + size_t(m.N) * m.s, 0.0);
    if (dvi) std::fill(dvi, dvi + size_t(m.N) * m.s, 0.0);
    for (size_t ii = prog.size(); ii-- > 0;) {
      const Op op = prog[ii];
      if (op == CR || op == CRDAG) {
        const bool dag = op == CRDAG;
        // group the stored input and the output adjoint by everything but b2
        std::map<Reg, std::pair<cplx, cplx>> xin, lout;
        for (auto& kv : stored[ii]) {
          Reg g = kv.first;
          const uint64_t b = g.b2;
          g.b2 = 0;
          (b ? xin[g].second : xin[g].first) = kv.second;
        }
        for (auto& kv : lam) {
          Reg g = kv.first;
          const uint64_t b = g.b2;
          g.b2 = 0;
          (b ? lout[g].second : lout[g].first) = kv.second;
        }
        for (auto& gv : xin) {
          auto it = lout.find(gv.first);
          if (it == lout.end()) continue;
          const Reg& g = gv.first;
          const double a = double_of(g.A), ai = double_of(g.A2);  // A2 = 0 for real matrices
          const cplx x0 = gv.second.first, x1 = gv.second.second;
          const cplx l0 = it->second.first, l1 = it->second.second;
          // 2 Re <lambda_out| dU/dp |x_in> for a real parameter p of the value
          const auto contrib = [&](const Rot& d) {
            cplx D[2][2];
            rot_matrix(d, dag, D);  // derivative of R or of R^dagger (p is real)
            const cplx y0 = D[0][0] * x0 + D[0][1] * x1;
            const cplx y1 = D[1][0] * x0 + D[1][1] * x1;
            return 2.0 * (std::conj(l0) * y0 + std::conj(l1) * y1).real();
          };
          const int32_t* row = &m.col[g.j * m.s];
          const uint64_t l = g.kc ^ qbs(row, m.s, g.k);
          if (l >= uint64_t(m.s)) fail("rotation site with slot >= s");
          if (bits_of(m.val[g.j * m.s + l]) != g.A) fail("A register does not hold a_{j,l}");
          if (!dvi) {
            dv[g.j * m.s + l] += contrib(rotation_deriv(a, g.j, g.k));
          } else {
            if (bits_of(m.vim[g.j * m.s + l]) != g.A2) fail("A2 register does not hold Im a_{j,l}");
            dv[g.j * m.s + l] += contrib(rotation_deriv_c(a, ai, g.j, g.k, false));
            dvi[g.j * m.s + l] += contrib(rotation_deriv_c(a, ai, g.j, g.k, true));
          }
        }
      }
      apply(lam, m, inverse(op));
    }
    std::fill(dbre, dbre + m.N, 0.0);
    std::fill(dbim, dbim + m.N, 0.0);
    for (auto& kv : lam) {
      const Reg& r = kv.first;
      if (r.jc == 0 && r.b1 == 0 && r.kc == 0 && r.k == 0 && r.b2 == 0 && r.A == 0 && r.A2 == 0) {
        dbre[r.j] = 2.0 * kv.second.real();
        dbim[r.j] = 2.0 * kv.second.imag();
      }
    }
  });
}

int orc_grad(void* mat, const double* bre, const double* bim, int32_t nb, int32_t nsteps, const double* w,
             double tau, double* dv, double* dbre, double* dbim, double* loss) {
  return grad_impl(mat, bre, bim, nb, nsteps, w, tau, dv, nullptr, dbre, dbim, loss);
}

// The complex matrices' form: dv = dL/dRe v, dvi = dL/dIm v by ELL slot.
int orc_grad_complex(void* mat, const double* bre, const double* bim, int32_t nb, int32_t nsteps, const double* w,
                     double tau, double* dv, double* dvi, double* dbre, double* dbim, double* loss) {
  if (!dvi) return guarded([] { fail("orc_grad_complex needs dvi"); });
  return grad_impl(mat, bre, bim, nb, nsteps, w, tau, dv, dvi, dbre, dbim, loss);
}

}  // extern "C"
