// CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow and deliberately literal CPU implementation of flexible
// CRC-aided successive-cancellation list (SCL) decoding of polar codes, as
// described in Leonardon, Cassagne, Leroux, Jego, Hamelin and Savaria,
// "Fast and Flexible Software Polar List Decoders" (arXiv:1710.08314).
//
// Only the test-suite, the smoke check and the CPU-baseline leg of the
// benchmark may load this library.  The product decoder (HIP, under the
// package directory) shares no code, header, table or generator with it.
//
// Structure, in the order of the paper:
//   * Sec. II-A: polar transform F^{(x)n} (footnote of Sec. II-A), frozen-set
//     construction by channel reliability, systematic encoding, CRC
//     concatenation (|A| = K + c).
//   * Sec. II-B1: f, g, h node updates (equations of Sec. II-B1).
//   * Sec. II-B2, Algorithm 1: recursive SCL_decode over the buffers
//     lambda[L][2N] and s_hat[L][N]; update_paths() at leaves; LLR-based
//     path metric (reference [balatsoukas2015llr] of the paper).
//   * Sec. II-B3: Rate-0 / Rate-1 / REP / SPC dedicated nodes (SSCL).
//   * Sec. II-B4: CRC-aided selection; Sec. IV-B: CRC checked in path-metric
//     order, first valid candidate wins.
//   * Sec. II-B5: fully / partially adaptive list size escalation.
//   * Sec. III-B3: 8-bit / 16-bit fixed point, saturation after every
//     operation, path-metric normalisation after every update_paths().
//
// Readings of points the paper leaves open are listed next to the code that
// takes them.  Parity status: every function here is pinned by the not-gpu
// tests (closed forms, brute-force ML, textbook reductions, invariances).
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fPIC -shared (no fast-math:
// the float32 mode must round exactly as written).

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Sec. II-A: code construction.
// ---------------------------------------------------------------------------

// Bhattacharyya parameters of the N synthetic channels, in the log domain.
// The paper names density evolution / Gaussian approximation (Sec. II-A,
// Sec. III-A) without fixing one; the reading taken here is the
// Bhattacharyya recursion: the index bits are read from the most significant
// (root split) to the least significant; a 0 bit is the "f" (worse) child,
// Z -> 2Z - Z^2, a 1 bit is the "g" (better) child, Z -> Z^2.  Exact for the
// binary erasure channel.
double log_bad_child(double lz) {
  // log(2Z - Z^2).  Two regimes so that neither small nor near-one Z loses
  // precision: 2Z - Z^2 = Z (2 - Z) = 1 - (1 - Z)^2.
  if (lz < -1.0) return lz + std::log(2.0 - std::exp(lz));
  double t = std::expm1(lz);  // Z - 1
  return std::log1p(-(t * t));
}

void logz_from_z0(int n, double lz0, double* out) {
  const int N = 1 << n;
  for (int i = 0; i < N; ++i) {
    double lz = lz0;
    for (int b = n - 1; b >= 0; --b) {
      if ((i >> b) & 1)
        lz = 2.0 * lz;
      else
        lz = log_bad_child(lz);
    }
    out[i] = lz;
  }
}

// ---------------------------------------------------------------------------
// Footnote of Sec. II-A: F^{(x)1} = [[1,0],[1,1]],
// F^{(x)n} = [[F^{(x)n-1}, 0], [F^{(x)n-1}, F^{(x)n-1}]], natural order.
// Row vector times matrix: x = v F^{(x)n}.  With v = (v_a, v_b) (halves):
// x = (v_a F' + v_b F', v_b F') over GF(2).
// ---------------------------------------------------------------------------
void transform_rec(const uint8_t* v, int N, uint8_t* x) {
  if (N == 1) {
    x[0] = v[0] & 1;
    return;
  }
  const int h = N / 2;
  std::vector<uint8_t> xa(h), xb(h);
  transform_rec(v, h, xa.data());
  transform_rec(v + h, h, xb.data());
  for (int i = 0; i < h; ++i) {
    x[i] = xa[i] ^ xb[i];
    x[h + i] = xb[i];
  }
}

// ---------------------------------------------------------------------------
// CRC (Sec. II-B4, Sec. IV-B).  Textbook bitwise long division of m(x) x^c
// by g(x): message bits most significant first, register initialised to 0,
// no reflection, no final xor.  `poly` holds the c low coefficients of g(x);
// a given x^c term (e.g. 0x1864CFB for c = 24) is masked away.
// ---------------------------------------------------------------------------
uint64_t crc_bits(const uint8_t* bits, int nbits, int c, uint64_t poly) {
  if (c == 0) return 0;
  const uint64_t mask = (c == 64) ? ~0ull : ((1ull << c) - 1);
  poly &= mask;
  uint64_t reg = 0;
  for (int i = 0; i < nbits; ++i) {
    uint64_t fb = ((reg >> (c - 1)) & 1ull) ^ (uint64_t)(bits[i] & 1);
    reg = (reg << 1) & mask;
    if (fb) reg ^= poly;
  }
  return reg;
}

// ---------------------------------------------------------------------------
// Value arithmetic.  Sec. II-B1 equations for f and g; Sec. III-B3 for the
// fixed-point modes (saturation after every operation).
//   Readings: hard decision HD(v) = [v < 0] by value, so +0 and -0 decide 0.
//   f's sign is that of the product, evaluated from the operand signs (so a
//   tiny product cannot underflow to a zero sign).  Saturation is symmetric:
//   int8 in [-127, 127], int16 in [-32767, 32767].  Node penalty sums are
//   exact in int32 and saturated once when added to the path metric; path
//   metrics live in [0, Q].  Float sums use the stride-halving order
//   v[i] += v[i + s], s = m/2 ... 1.
// ---------------------------------------------------------------------------
template <class T>
struct FloatArith {
  using V = T;    // LLR
  using P = T;    // path metric
  using Acc = T;  // penalty accumulator
  static constexpr bool kInt = false;
  static V f(V a, V b) {
    V mag = std::min(std::fabs(a), std::fabs(b));
    bool neg = (a < 0) != (b < 0);
    return neg ? -mag : mag;
  }
  static V g(V a, V b, int s) { return s ? (b - a) : (b + a); }
  static bool hd(V v) { return v < 0; }
  static Acc mag(V v) { return std::fabs(v); }
  static P pm_add(P pm, Acc pen) { return pm + pen; }
  static V known() { return (V)1048576.0; }  // 2^20: finite, no inf-inf in g
  static double as_double(P p) { return (double)p; }
};

template <class T, int Q>
struct IntArith {
  using V = T;
  using P = int32_t;
  using Acc = int32_t;
  static constexpr bool kInt = true;
  static V sat(int32_t v) { return (V)std::max(-Q, std::min(Q, v)); }
  static V f(V a, V b) {
    int32_t ma = std::abs((int32_t)a), mb = std::abs((int32_t)b);
    int32_t mag = std::min(ma, mb);
    bool neg = (a < 0) != (b < 0);
    return (V)(neg ? -mag : mag);
  }
  static V g(V a, V b, int s) {
    return sat(s ? ((int32_t)b - (int32_t)a) : ((int32_t)b + (int32_t)a));
  }
  static bool hd(V v) { return v < 0; }
  static Acc mag(V v) { return std::abs((int32_t)v); }
  static P pm_add(P pm, Acc pen) { return std::min<int64_t>((int64_t)pm + pen, Q); }
  static V known() { return (V)Q; }
  static double as_double(P p) { return (double)p; }
};

using F32 = FloatArith<float>;
using F64 = FloatArith<double>;
using I16 = IntArith<int16_t, 32767>;
using I8 = IntArith<int8_t, 127>;

template <class Acc>
Acc sum_stride_halving(std::vector<Acc> v) {
  size_t m = v.size();
  if (m == 0) return Acc(0);
  for (size_t s = m / 2; s >= 1; s /= 2) {
    for (size_t i = 0; i < s; ++i) v[i] = v[i] + v[i + s];
  }
  return v[0];
}

}  // namespace

// ---------------------------------------------------------------------------
// Public C interface (ctypes).
// ---------------------------------------------------------------------------
extern "C" {

enum { ORC_F32 = 0, ORC_I16 = 1, ORC_I8 = 2, ORC_F64 = 3 };
enum { ORC_SC = 0, ORC_CA_SCL = 1, ORC_PA_SCL = 2, ORC_FA_SCL = 3 };
enum { ORC_NODE_R0 = 1, ORC_NODE_R1 = 2, ORC_NODE_REP = 4, ORC_NODE_SPC = 8 };
enum { K_LEAF_F = 0, K_LEAF_I = 1, K_R0 = 2, K_R1 = 3, K_REP = 4, K_SPC = 5, K_SPLIT = 6 };

typedef struct {
  int32_t N;            // mother code length (power of two)
  int32_t K;            // |A|, information positions INCLUDING the c CRC bits
  int32_t crc_len;      // c (0 = no CRC)
  uint64_t crc_poly;    // c low coefficients of g(x)
  const uint8_t* frozen;  // N bytes, 1 = frozen u-index
  int32_t S;            // shortened: codeword positions [N-S, N) known zero
  int32_t quant;        // ORC_F32 / ORC_I16 / ORC_I8 / ORC_F64
  int32_t algo;         // ORC_SC / ORC_CA_SCL / ORC_PA_SCL / ORC_FA_SCL
  int32_t L;            // list size (CA-SCL)
  int32_t L_max;        // largest list size (PA / FA)
  int32_t node_enable;  // OR of ORC_NODE_*
  int32_t rep_max, spc_max, r1_max, r0_max;  // 0 = unlimited node size
  int32_t P;            // punctured: codeword positions [0, P) not sent (LLR 0)
} orc_cfg;

typedef struct {
  int32_t crc_ok;    // 1 = the output passed the CRC (or there is no CRC)
  int32_t L_used;    // list size of the stage whose output was taken
  int32_t near_tie;  // float modes: a decision gap within 1e-4 relative
  int32_t n_pm;      // number of paths alive at the end of that stage
  double pm;         // path metric of the output path
} orc_status;

void orc_logz_z0(int n, double lz0, double* out) { logz_from_z0(n, lz0, out); }

// Frozen set: the N - |A| least reliable u-indices are frozen, i.e. |A| most
// reliable kept, ranked by (log Z ascending, index descending).  Shortened
// u-indices [N-S, N) and punctured u-indices [0, P) are frozen first: x_j
// is the XOR of the u_i with i a bitwise superset of j, so [N-S, N) (an
// up-set) carries only known zeros and, with x_[0,P) (a down-set) not sent,
// u_[0,P) cannot be recovered.  Design point: Eb/N0 in dB with
// R = (K - c) / (N - S - P) and Z0 = exp(-R Eb/N0).  Returns 0, or -1 on bad
// args.
int orc_construct_lz0p(int N, int K, int S, int P, double lz0, uint8_t* frozen) {
  int n = 0;
  while ((1 << n) < N) ++n;
  if ((1 << n) != N || K < 0 || S < 0 || P < 0 || K > N - S - P) return -1;
  std::vector<double> lz(N);
  logz_from_z0(n, lz0, lz.data());
  std::vector<int> idx;
  for (int i = P; i < N - S; ++i) idx.push_back(i);
  std::sort(idx.begin(), idx.end(), [&](int a, int b) {
    if (lz[a] != lz[b]) return lz[a] < lz[b];
    return a > b;
  });
  for (int i = 0; i < N; ++i) frozen[i] = 1;
  for (int j = 0; j < K; ++j) frozen[idx[j]] = 0;
  return 0;
}

int orc_construct_lz0(int N, int K, int S, double lz0, uint8_t* frozen) {
  return orc_construct_lz0p(N, K, S, 0, lz0, frozen);
}

int orc_construct_p(int N, int K, int S, int P, int crc_len, double design_ebn0_db,
                    uint8_t* frozen) {
  if (N - S - P <= 0) return -1;
  const double rate = (double)(K - crc_len) / (double)(N - S - P);
  return orc_construct_lz0p(N, K, S, P, -rate * std::pow(10.0, design_ebn0_db / 10.0), frozen);
}

int orc_construct(int N, int K, int S, int crc_len, double design_ebn0_db, uint8_t* frozen) {
  return orc_construct_p(N, K, S, 0, crc_len, design_ebn0_db, frozen);
}

// f (op 0) or g (op 1, partial sum s) of the given mode on one pair, for the
// truth-table tests; values are passed and returned as double.
double orc_fg(int quant, int op, double a, double b, int s) {
  switch (quant) {
    case ORC_F32: return op ? F32::g((float)a, (float)b, s) : F32::f((float)a, (float)b);
    case ORC_I16:
      return op ? I16::g((int16_t)a, (int16_t)b, s) : I16::f((int16_t)a, (int16_t)b);
    case ORC_I8: return op ? I8::g((int8_t)a, (int8_t)b, s) : I8::f((int8_t)a, (int8_t)b);
    default: return op ? F64::g(a, b, s) : F64::f(a, b);
  }
}

void orc_transform(int N, const uint8_t* v, uint8_t* x) { transform_rec(v, N, x); }

// Systematic encoding (Sec. II-A): b -> u_A (ascending index), u' = u F,
// u'_{A^c} = 0, x = u' F.
void orc_encode(int N, const uint8_t* frozen, const uint8_t* b, uint8_t* x) {
  std::vector<uint8_t> u(N, 0), up(N);
  int j = 0;
  for (int i = 0; i < N; ++i)
    if (!frozen[i]) u[i] = b[j++] & 1;
  transform_rec(u.data(), N, up.data());
  for (int i = 0; i < N; ++i)
    if (frozen[i]) up[i] = 0;
  transform_rec(up.data(), N, x);
}

uint64_t orc_crc(const uint8_t* bits, int nbits, int c, uint64_t poly) {
  return crc_bits(bits, nbits, c, poly);
}

// b = data || CRC(data), the c CRC bits most significant first (Sec. II-B4).
void orc_attach_crc(const uint8_t* data, int kd, int c, uint64_t poly, uint8_t* b) {
  for (int i = 0; i < kd; ++i) b[i] = data[i] & 1;
  uint64_t r = crc_bits(data, kd, c, poly);
  for (int t = 0; t < c; ++t) b[kd + t] = (uint8_t)((r >> (c - 1 - t)) & 1ull);
}

// Channel of the Monte-Carlo chain (Sec. II-C): BPSK 0 -> +1, 1 -> -1,
// y = s + sigma n, LLR = 2 y / sigma^2.  `noise` holds standard normals.
void orc_bpsk_awgn_llr(const uint8_t* x, int n, const double* noise, double sigma, double* llr) {
  const double s2 = sigma * sigma;
  for (int i = 0; i < n; ++i) {
    double s = x[i] ? -1.0 : 1.0;
    double y = s + sigma * noise[i];
    llr[i] = 2.0 * y / s2;
  }
}

// Sec. III-B3 LLR quantisation.  Reading: q = clamp(rint(l 2^frac), -Q, Q),
// round half to even; float32 mode: nearest float.
void orc_quantize(const double* llr, int n, int quant, int frac, void* out) {
  const double scale = std::ldexp(1.0, frac);
  for (int i = 0; i < n; ++i) {
    if (quant == ORC_F32) {
      ((float*)out)[i] = (float)llr[i];
    } else if (quant == ORC_F64) {
      ((double*)out)[i] = llr[i];
    } else {
      const double Q = quant == ORC_I8 ? 127.0 : 32767.0;
      double q = std::nearbyint(llr[i] * scale);
      q = std::max(-Q, std::min(Q, q));
      if (quant == ORC_I8)
        ((int8_t*)out)[i] = (int8_t)q;
      else
        ((int16_t*)out)[i] = (int16_t)q;
    }
  }
}

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Sec. II-B3 dedicated nodes.  Node [start, start+m) of the u-vector is
//   R0  : every leaf frozen;
//   R1  : every leaf information;
//   REP : every leaf frozen except the last;
//   SPC : only the first leaf frozen (m >= 4);
// each enabled separately and limited in size (Sec. III-B2: SPC4 / SPC4+,
// REP8-).  Reading of the precedence: R0, R1, REP, SPC; a size-2 node
// [frozen, info] is REP.  Size-1 nodes are plain leaves.
// ---------------------------------------------------------------------------
int classify(const orc_cfg& c, int start, int m) {
  if (m == 1) return c.frozen[start] ? K_LEAF_F : K_LEAF_I;
  int nf = 0;
  for (int i = 0; i < m; ++i) nf += c.frozen[start + i] ? 1 : 0;
  auto fits = [](int lim, int m) { return lim == 0 || m <= lim; };
  if ((c.node_enable & ORC_NODE_R0) && nf == m && fits(c.r0_max, m)) return K_R0;
  if ((c.node_enable & ORC_NODE_R1) && nf == 0 && fits(c.r1_max, m)) return K_R1;
  if ((c.node_enable & ORC_NODE_REP) && nf == m - 1 && !c.frozen[start + m - 1] &&
      fits(c.rep_max, m))
    return K_REP;
  if ((c.node_enable & ORC_NODE_SPC) && m >= 4 && nf == 1 && c.frozen[start] &&
      fits(c.spc_max, m))
    return K_SPC;
  return K_SPLIT;
}

// ---------------------------------------------------------------------------
// Algorithm 1 (Sec. II-B2) with the dedicated nodes of Sec. II-B3.
//   lambda[p][2N], s_hat[p][N] exactly as the algorithm's buffers: the node
//   of size m at LLR offset o_l has its child at o_l + m; f and g write the
//   child; the left child's partial sums land in [o_s, o_s + m/2), the right
//   child's in [o_s + m/2, o_s + m), and h combines them in place.
//   update_paths(): every candidate's metric is PM + penalty, the penalty
//   being the sum of |alpha_i| over positions whose decision disagrees with
//   HD(alpha_i) (LLR-based metric with the min-sum approximation).  Paths are
//   duplicated by copying their whole buffers.
// ---------------------------------------------------------------------------
template <class A>
class Scl {
 public:
  using V = typename A::V;
  using P = typename A::P;
  using Acc = typename A::Acc;

  Scl(const orc_cfg& cfg, int L) : c_(cfg), N_(cfg.N), L_(L) {
    lam_.assign(L_, std::vector<V>(2 * N_, V(0)));
    s_.assign(L_, std::vector<uint8_t>(N_, 0));
    pm_.assign(L_, P(0));
  }

  // Decode one frame from N channel LLRs (shortened positions already set).
  void run(const std::vector<V>& chan) {
    a_ = 1;
    pm_[0] = P(0);
    near_tie_ = false;
    for (int i = 0; i < N_; ++i) lam_[0][i] = chan[i];
    decode(N_, 0, 0);
  }

  // Sec. II-B4 / Sec. IV-B: candidates ordered by (path metric, rank); the
  // first one whose information part passes the CRC is the decision; if none
  // passes, the best metric (crc_ok = 0).  `out_info` gets b_hat = x_hat_A.
  void select(std::vector<uint8_t>& b_hat, std::vector<uint8_t>& x_hat, bool& crc_ok,
              P& pm_out, std::vector<double>& pm_list) {
    std::vector<int> ord(a_);
    for (int i = 0; i < a_; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return pm_[x] < pm_[y]; });
    pm_list.clear();
    for (int i = 0; i < a_; ++i) pm_list.push_back(A::as_double(pm_[ord[i]]));
    const int K = c_.K, cl = c_.crc_len;
    int chosen = -1, chosen_pos = -1;
    std::vector<uint8_t> b(K);
    for (int pos = 0; pos < a_ && chosen < 0; ++pos) {
      int p = ord[pos];
      extract(p, b);
      if (cl == 0 || crc_bits(b.data(), K - cl, cl, c_.crc_poly) == tail_value(b)) {
        chosen = p;
        chosen_pos = pos;
      }
    }
    crc_ok = chosen >= 0;
    if (!crc_ok) {
      chosen = ord[0];
      chosen_pos = 0;
    }
    // near-tie: the chosen path's metric within 1e-4 relative of a path that
    // also passes the CRC (or of the runner-up when nothing passes).
    if (!A::kInt) {
      for (int pos = 0; pos < a_; ++pos) {
        if (pos == chosen_pos) continue;
        int p = ord[pos];
        extract(p, b);
        bool ok = cl == 0 || crc_bits(b.data(), K - cl, cl, c_.crc_poly) == tail_value(b);
        if (!crc_ok || ok) {
          double d = std::fabs(A::as_double(pm_[p]) - A::as_double(pm_[chosen]));
          if (d <= 1e-4 * std::max(1.0, std::fabs(A::as_double(pm_[chosen])))) near_tie_ = true;
        }
      }
    }
    extract(chosen, b);
    b_hat.assign(b.begin(), b.begin() + (K - cl));
    x_hat.assign(s_[chosen].begin(), s_[chosen].end());
    pm_out = pm_[chosen];
  }

  int alive() const { return a_; }
  bool near_tie() const { return near_tie_; }

 private:
  uint64_t tail_value(const std::vector<uint8_t>& b) const {
    uint64_t r = 0;
    for (int t = 0; t < c_.crc_len; ++t) r = (r << 1) | b[c_.K - c_.crc_len + t];
    return r;
  }
  // b_hat = x_hat_A: the codeword bits at the information positions, in
  // ascending order (systematic code, Sec. II-A / Sec. IV-B).
  void extract(int p, std::vector<uint8_t>& b) const {
    int j = 0;
    for (int i = 0; i < N_; ++i)
      if (!c_.frozen[i]) b[j++] = s_[p][i];
  }

  void decode(int m, int ol, int os) {
    int kind = classify(c_, os, m);
    if (kind != K_SPLIT) {
      update_paths(kind, m, ol, os);
      return;
    }
    const int h = m / 2;
    for (int p = 0; p < a_; ++p)
      for (int i = 0; i < h; ++i) lam_[p][ol + m + i] = A::f(lam_[p][ol + i], lam_[p][ol + h + i]);
    decode(h, ol + m, os);
    for (int p = 0; p < a_; ++p)
      for (int i = 0; i < h; ++i)
        lam_[p][ol + m + i] = A::g(lam_[p][ol + i], lam_[p][ol + h + i], s_[p][os + i]);
    decode(h, ol + m, os + h);
    for (int p = 0; p < a_; ++p)
      for (int i = 0; i < h; ++i) s_[p][os + i] = s_[p][os + i] ^ s_[p][os + h + i];
  }

  struct Cand {
    P pm;
    int parent;
    int local;
    std::vector<uint8_t> beta;
  };

  // sum over k of |alpha_k| [HD(alpha_k) != v], stride-halving order
  Acc disagree_sum(const V* al, int m, int v) const {
    std::vector<Acc> t(m);
    for (int k = 0; k < m; ++k) t[k] = ((int)A::hd(al[k]) != v) ? A::mag(al[k]) : Acc(0);
    return sum_stride_halving(t);
  }

  void normalise() {
    if (!A::kInt || a_ == 0) return;
    P mn = pm_[0];
    for (int p = 1; p < a_; ++p) mn = std::min(mn, pm_[p]);
    for (int p = 0; p < a_; ++p) pm_[p] = pm_[p] - mn;
  }

  void update_paths(int kind, int m, int ol, int os) {
    // Single-candidate nodes (frozen leaf, R0): metric update in place,
    // ranks unchanged, decision 0.
    if (kind == K_LEAF_F || kind == K_R0) {
      for (int p = 0; p < a_; ++p) {
        Acc pen = disagree_sum(&lam_[p][ol], m, 0);
        pm_[p] = A::pm_add(pm_[p], pen);
        for (int i = 0; i < m; ++i) s_[p][os + i] = 0;
      }
      normalise();
      return;
    }
    std::vector<Cand> cands;
    for (int p = 0; p < a_; ++p) {
      const V* al = &lam_[p][ol];
      std::vector<uint8_t> hdv(m);
      for (int k = 0; k < m; ++k) hdv[k] = A::hd(al[k]) ? 1 : 0;
      if (kind == K_LEAF_I || kind == K_REP) {
        // two candidates: all-0 and all-1 (for a leaf, the bit itself)
        for (int v = 0; v < 2; ++v) {
          Cand cd{A::pm_add(pm_[p], disagree_sum(al, m, v)), p, v,
                  std::vector<uint8_t>(m, (uint8_t)v)};
          cands.push_back(std::move(cd));
        }
      } else {
        // R1: Chase-2 over the 2 least reliable positions (the paper's
        // "two maximum absolute values" read as the two smallest |alpha|,
        // which is what a Chase-2 search flips).  SPC: the T = min(m, 4)
        // least reliable positions, masks whose weight has the parity of
        // HD(alpha), so that every candidate satisfies the parity check.
        std::vector<int> ord(m);
        for (int k = 0; k < m; ++k) ord[k] = k;
        std::sort(ord.begin(), ord.end(), [&](int x, int y) {
          Acc mx = A::mag(al[x]), my = A::mag(al[y]);
          if (mx != my) return mx < my;
          return x < y;
        });
        const int T = (kind == K_R1) ? 2 : std::min(m, 4);
        int parity = 0;
        for (int k = 0; k < m; ++k) parity ^= hdv[k];
        for (int mask = 0; mask < (1 << T); ++mask) {
          if (kind == K_SPC && (__builtin_popcount(mask) & 1) != parity) continue;
          Acc pen = Acc(0);
          std::vector<uint8_t> beta = hdv;
          for (int j = 0; j < T; ++j) {
            if ((mask >> j) & 1) {
              pen = pen + A::mag(al[ord[j]]);
              beta[ord[j]] ^= 1;
            }
          }
          Cand cd{A::pm_add(pm_[p], pen), p, mask, std::move(beta)};
          cands.push_back(std::move(cd));
        }
      }
    }
    std::stable_sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) {
      if (x.pm != y.pm) return x.pm < y.pm;
      if (x.parent != y.parent) return x.parent < y.parent;
      return x.local < y.local;
    });
    const int keep = std::min<int>(L_, (int)cands.size());
    if (!A::kInt && (int)cands.size() > keep && keep > 0) {
      double lo = A::as_double(cands[keep - 1].pm), hi = A::as_double(cands[keep].pm);
      if (hi - lo <= 1e-4 * std::max(1.0, std::fabs(lo))) near_tie_ = true;
    }
    std::vector<std::vector<V>> nl(keep);
    std::vector<std::vector<uint8_t>> ns(keep);
    std::vector<P> npm(keep);
    for (int i = 0; i < keep; ++i) {
      const Cand& cd = cands[i];
      nl[i] = lam_[cd.parent];
      ns[i] = s_[cd.parent];
      for (int k = 0; k < m; ++k) ns[i][os + k] = cd.beta[k];
      npm[i] = cd.pm;
    }
    for (int i = 0; i < keep; ++i) {
      lam_[i] = std::move(nl[i]);
      s_[i] = std::move(ns[i]);
      pm_[i] = npm[i];
    }
    a_ = keep;
    normalise();
  }

  const orc_cfg& c_;
  int N_, L_;
  int a_ = 1;
  bool near_tie_ = false;
  std::vector<std::vector<V>> lam_;
  std::vector<std::vector<uint8_t>> s_;
  std::vector<P> pm_;
};

// Sec. II-B5: list-size schedule of the decoding stages.
std::vector<int> stage_schedule(const orc_cfg& c) {
  std::vector<int> st;
  switch (c.algo) {
    case ORC_SC:
      st.push_back(1);
      break;
    case ORC_CA_SCL:
      st.push_back(c.L);
      break;
    case ORC_PA_SCL:
      st.push_back(1);
      if (c.L_max > 1) st.push_back(c.L_max);
      break;
    case ORC_FA_SCL:
    default: {
      int l = 1;
      while (l < c.L_max) {
        st.push_back(l);
        l *= 2;
      }
      st.push_back(c.L_max);
      break;
    }
  }
  return st;
}

template <class A>
int decode_frame(const orc_cfg& c, const void* llr_in, uint8_t* info_out, uint8_t* xhat_out,
                 double* pm_list_out, orc_status* st) {
  using V = typename A::V;
  const int N = c.N, P = c.P, Ntx = c.N - c.S - c.P;
  std::vector<V> chan(N);
  const V* src = (const V*)llr_in;
  for (int i = 0; i < P; ++i) chan[i] = V(0);  // punctured: nothing received
  for (int i = 0; i < Ntx; ++i) chan[P + i] = src[i];
  for (int i = P + Ntx; i < N; ++i) chan[i] = A::known();  // shortened: known zero bit
  std::vector<int> stages = stage_schedule(c);
  std::vector<uint8_t> b_hat, x_hat;
  std::vector<double> pm_list;
  bool ok = false, tie = false;
  typename A::P pm = 0;
  int used = 0, alive = 0;
  for (size_t si = 0; si < stages.size(); ++si) {
    Scl<A> dec(c, stages[si]);
    dec.run(chan);
    dec.select(b_hat, x_hat, ok, pm, pm_list);
    // near-tie over every stage run: a tie in a stage that failed its CRC
    // could have decided that failure, and with it the later stages
    tie = tie || dec.near_tie();
    used = stages[si];
    alive = dec.alive();
    if (ok) break;
  }
  std::memcpy(info_out, b_hat.data(), b_hat.size());
  if (xhat_out) std::memcpy(xhat_out, x_hat.data(), x_hat.size());
  if (pm_list_out)
    for (size_t i = 0; i < pm_list.size(); ++i) pm_list_out[i] = pm_list[i];
  st->crc_ok = ok ? 1 : 0;
  st->L_used = used;
  st->near_tie = tie ? 1 : 0;
  st->n_pm = alive;
  st->pm = A::as_double(pm);
  return 0;
}

int check_cfg(const orc_cfg* c) {
  if (!c || !c->frozen) return -1;
  int n = 0;
  while ((1 << n) < c->N) ++n;
  if (c->N < 1 || (1 << n) != c->N) return -1;
  if (c->S < 0 || c->P < 0 || c->S + c->P >= c->N) return -1;
  int na = 0;
  for (int i = 0; i < c->N; ++i) na += c->frozen[i] ? 0 : 1;
  if (na != c->K || c->crc_len < 0 || c->crc_len > 64 || c->crc_len > c->K) return -1;
  for (int i = c->N - c->S; i < c->N; ++i)
    if (!c->frozen[i]) return -1;
  for (int i = 0; i < c->P; ++i)
    if (!c->frozen[i]) return -1;
  if (c->algo == ORC_CA_SCL && c->L < 1) return -1;
  if ((c->algo == ORC_PA_SCL || c->algo == ORC_FA_SCL) && (c->L_max < 1 || c->crc_len == 0))
    return -1;
  if (c->quant < ORC_F32 || c->quant > ORC_F64) return -1;
  return 0;
}

size_t elem_size(int quant) {
  switch (quant) {
    case ORC_F32: return 4;
    case ORC_I16: return 2;
    case ORC_I8: return 1;
    default: return 8;
  }
}

int decode_any(const orc_cfg* c, const void* llr, uint8_t* info, uint8_t* xhat, double* pml,
               orc_status* st) {
  switch (c->quant) {
    case ORC_F32: return decode_frame<F32>(*c, llr, info, xhat, pml, st);
    case ORC_I16: return decode_frame<I16>(*c, llr, info, xhat, pml, st);
    case ORC_I8: return decode_frame<I8>(*c, llr, info, xhat, pml, st);
    default: return decode_frame<F64>(*c, llr, info, xhat, pml, st);
  }
}

int max_list(const orc_cfg* c) {
  int m = 1;
  for (int l : stage_schedule(*c)) m = std::max(m, l);
  return m;
}

}  // namespace

extern "C" {

// Batch helpers of the Monte-Carlo chain (test-input generation): frame f
// has kd data bits data[f * kd ...], gets b = data || CRC, the systematic
// codeword, then BPSK/AWGN LLRs of its sent positions [P, N - S) quantised
// to the mode (noise[f * ntx ...] standard normals, ntx = N - S - P).
// `out` holds ntx values of the mode per frame.
int orc_make_frames(const orc_cfg* c, int n, const uint8_t* data, const double* noise,
                    double sigma, int frac, void* out) {
  const int N = c->N, ntx = c->N - c->S - c->P, kd = c->K - c->crc_len;
  std::vector<uint8_t> b(c->K), x(N);
  std::vector<double> l(ntx);
  const size_t es = elem_size(c->quant);
  for (int f = 0; f < n; ++f) {
    orc_attach_crc(data + (size_t)f * kd, kd, c->crc_len, c->crc_poly, b.data());
    orc_encode(N, c->frozen, b.data(), x.data());
    orc_bpsk_awgn_llr(x.data() + c->P, ntx, noise + (size_t)f * ntx, sigma, l.data());
    orc_quantize(l.data(), ntx, c->quant, frac, (char*)out + (size_t)f * ntx * es);
  }
  return 0;
}

// Decode one frame.  `llr` holds N - S values of the mode's type (float,
// int16, int8 or double), natural codeword order.  `info` receives K - c
// bytes (0/1); `xhat` (nullable) N bytes; `pm_list` (nullable) up to the
// largest list size of the schedule, sorted ascending.
int orc_decode(const orc_cfg* cfg, const void* llr, uint8_t* info, uint8_t* xhat,
               double* pm_list, orc_status* st) {
  int rc = check_cfg(cfg);
  if (rc) return rc;
  return decode_any(cfg, llr, info, xhat, pm_list, st);
}

// Decode `n` frames with `threads` host threads (frames are independent; each
// frame is decoded by one thread exactly as orc_decode does).  Frame f reads
// llr + f * llr_stride_bytes and writes info + f * (K - c), xhat + f * N,
// pm_list + f * max list size, st + f.  Returns 0 or the first error.
int orc_decode_batch(const orc_cfg* cfg, int n, const void* llr, int64_t llr_stride_bytes,
                     uint8_t* info, uint8_t* xhat, double* pm_list, orc_status* st, int threads) {
  int rc = check_cfg(cfg);
  if (rc) return rc;
  const int kd = cfg->K - cfg->crc_len;
  const int lm = max_list(cfg);
  std::atomic<int> next(0);
  auto worker = [&]() {
    for (;;) {
      int f = next.fetch_add(1);
      if (f >= n) break;
      decode_any(cfg, (const char*)llr + (int64_t)f * llr_stride_bytes, info + (int64_t)f * kd,
                 xhat ? xhat + (int64_t)f * cfg->N : nullptr,
                 pm_list ? pm_list + (int64_t)f * lm : nullptr, st + f);
    }
  };
  if (threads <= 1) {
    worker();
  } else {
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t) pool.emplace_back(worker);
    for (auto& t : pool) t.join();
  }
  return 0;
}

// The dedicated-node decomposition the decoder walks, in pre-order: for each
// node, kind (0 frozen leaf, 1 info leaf, 2 R0, 3 R1, 4 REP, 5 SPC), first
// leaf index and size.  Returns the number of nodes written (<= cap).
int orc_nodes(const orc_cfg* c, int32_t* kind, int32_t* start, int32_t* size, int cap) {
  int cnt = 0;
  struct Rec {
    static void go(const orc_cfg* c, int s, int m, int32_t* k, int32_t* st, int32_t* sz,
                   int cap, int& cnt) {
      int t = classify(*c, s, m);
      if (t == K_SPLIT) {
        go(c, s, m / 2, k, st, sz, cap, cnt);
        go(c, s + m / 2, m / 2, k, st, sz, cap, cnt);
        return;
      }
      if (cnt < cap) {
        k[cnt] = t;
        st[cnt] = s;
        sz[cnt] = m;
      }
      ++cnt;
    }
  };
  Rec::go(c, 0, c->N, kind, start, size, cap, cnt);
  return cnt;
}

size_t orc_elem_size(int quant) { return elem_size(quant); }

}  // extern "C"
