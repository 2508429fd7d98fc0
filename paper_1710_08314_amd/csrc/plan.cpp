// Host planner of the polar SCL decoder: everything that depends only on the
// code and decoder parameters (Sec. III-A genericity, Sec. III-B flexibility),
// computed once per plan and uploaded as a device blob.
//
//   * frozen set by the Bhattacharyya recursion (reading of Sec. II-A, which
//     names reliability ordering without fixing a method or design point);
//   * check that the systematic encoder of Sec. II-A gives x_A = b;
//   * the pruned decoding tree (Sec. II-B3) as a pre-order node program;
//   * CRC syndrome columns so that a path's CRC is checked straight from its
//     codeword estimate, without first extracting the information bits
//     (Sec. IV-B: packed words and precomputed sub-results);
//   * the LDS footprint of one frame at each list size.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace polar {

namespace {

uint32_t ilog2(uint32_t x) {
  uint32_t n = 0;
  while ((1u << n) < x) ++n;
  return n;
}

bool is_pow2(uint32_t x) { return x && !(x & (x - 1)); }

// log Z of the "f" child: log(2Z - Z^2), computed as log Z + log(2 - Z) for
// small Z and as log1p(-(1 - Z)^2) near Z = 1.
double lz_minus(double lz) {
  if (lz < -1.0) return lz + std::log(2.0 - std::exp(lz));
  const double t = std::expm1(lz);
  return std::log1p(-(t * t));
}

// Polar transform x = v F^{(x)n} on packed bits, in place (bw words hold N
// bits).  Each butterfly stage XORs the second half of every block of size
// 2s into its first half; the stages commute.
void transform_words(std::vector<uint32_t>& w, uint32_t N) {
  static const uint32_t kMask[5] = {0x55555555u, 0x33333333u, 0x0F0F0F0Fu, 0x00FF00FFu,
                                    0x0000FFFFu};
  for (uint32_t s = 1, k = 0; s < N && s < 32; s <<= 1, ++k)
    for (auto& x : w) x ^= (x >> s) & kMask[k];
  for (uint32_t S = 1; 32 * S < N; S <<= 1)
    for (uint32_t i = 0; i < w.size(); ++i)
      if (!(i & S)) w[i] ^= w[i + S];
}

inline bool bit(const std::vector<uint32_t>& w, uint32_t j) { return (w[j >> 5] >> (j & 31)) & 1u; }

// The move masks of a five-step bit compress (H. S. Warren, Hacker's
// Delight, Sec. 7-4): step i shifts the bits of mv[i] down by 2^i, and the
// five steps together gather the bits of a word at the set positions of m,
// in order, to the low end.  A bit moves at step i when bit i of the count
// of zeros of m below it is set; mk holds those counts' parity one bit at a
// time, taken as a prefix XOR.
void compress_masks(uint32_t m, uint32_t mv[5]) {
  uint32_t mk = ~m << 1;
  for (int i = 0; i < 5; ++i) {
    uint32_t mp = mk ^ (mk << 1);
    mp ^= mp << 2;
    mp ^= mp << 4;
    mp ^= mp << 8;
    mp ^= mp << 16;
    const uint32_t v = mp & m;
    m = (m ^ v) | (v >> (1u << i));
    mk &= ~mp;
    mv[i] = v;
  }
}

}  // namespace

std::vector<double> bhattacharyya_log(uint32_t n, double lz0) {
  const uint32_t N = 1u << n;
  std::vector<double> out(N);
  // breadth-first over the tree levels: level k holds 2^k values
  std::vector<double> cur{lz0};
  for (uint32_t k = 0; k < n; ++k) {
    std::vector<double> nxt(cur.size() * 2);
    for (size_t i = 0; i < cur.size(); ++i) {
      nxt[2 * i] = lz_minus(cur[i]);      // next index bit 0
      nxt[2 * i + 1] = 2.0 * cur[i];      // next index bit 1
    }
    cur.swap(nxt);
  }
  // cur[i] walks the index bits from the most significant: i is the index
  for (uint32_t i = 0; i < N; ++i) out[i] = cur[i];
  return out;
}

int make_plan(const polar_plan_desc& d, HostPlan& hp) {
  if (d.N < 2 || d.N > kMaxN || !is_pow2(d.N)) return d.N > kMaxN && is_pow2(d.N) ? POLAR_EUNSUP : POLAR_EINVAL;
  const uint32_t N = d.N, n = ilog2(N), S = d.n_shorten, Pn = d.n_puncture;
  if (S >= N || Pn >= N - S || d.K == 0 || d.K > N - S - Pn) return POLAR_EINVAL;
  if (d.crc_len > 32) return POLAR_EUNSUP;
  if (d.crc_len >= d.K) return POLAR_EINVAL;
  if (d.quant > POLAR_I8 || d.algo > POLAR_FA_SCL) return POLAR_EINVAL;
  uint32_t first = 1, maxl = 1;
  switch (d.algo) {
    case POLAR_SC: first = maxl = 1; break;
    case POLAR_CA_SCL:
      if (!is_pow2(d.L)) return POLAR_EINVAL;
      if (d.L > kMaxL) return POLAR_EUNSUP;
      first = maxl = d.L;
      break;
    default:
      if (!is_pow2(d.L_max) || d.crc_len == 0) return POLAR_EINVAL;
      if (d.L_max > kMaxL) return POLAR_EUNSUP;
      first = 1;
      maxl = d.L_max;
      break;
  }
  const uint32_t bw = N >= 32 ? N / 32 : 1;

  // ---- frozen set
  std::vector<uint32_t> frozen(bw, 0);
  if (d.frozen) {
    for (uint32_t w = 0; w < bw; ++w) frozen[w] = d.frozen[w];
    if (N < 32) frozen[0] &= (1u << N) - 1;
    uint32_t na = 0;
    for (uint32_t j = 0; j < N; ++j) na += bit(frozen, j) ? 0 : 1;
    if (na != d.K) return POLAR_EINVAL;
    for (uint32_t j = N - S; j < N; ++j)
      if (!bit(frozen, j)) return POLAR_EINVAL;
    for (uint32_t j = 0; j < Pn; ++j)
      if (!bit(frozen, j)) return POLAR_EINVAL;
  } else {
    // rate over the sent positions; shortened u-indices [N-S, N) (their bits
    // are known zeros) and punctured u-indices [0, P) (their bits reach only
    // unsent positions) are frozen before ranking the rest
    const double rate = double(d.K - d.crc_len) / double(N - S - Pn);
    const double lz0 = -rate * std::pow(10.0, double(d.design_ebn0_db) / 10.0);
    std::vector<double> lz = bhattacharyya_log(n, lz0);
    std::vector<uint32_t> idx(N - S - Pn);
    std::iota(idx.begin(), idx.end(), Pn);
    // most reliable first: smaller log Z, ties to the larger index
    std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) {
      return lz[a] < lz[b] || (lz[a] == lz[b] && a > b);
    });
    for (uint32_t w = 0; w < bw; ++w) frozen[w] = ~0u;
    if (N < 32) frozen[0] = (1u << N) - 1;
    for (uint32_t k = 0; k < d.K; ++k) frozen[idx[k] >> 5] &= ~(1u << (idx[k] & 31));
  }
  std::vector<uint32_t> info(bw);
  for (uint32_t w = 0; w < bw; ++w) info[w] = ~frozen[w];
  if (N < 32) info[0] &= (1u << N) - 1;
  std::vector<uint32_t> A;
  for (uint32_t j = 0; j < N; ++j)
    if (bit(info, j)) A.push_back(j);

  // ---- systematic check: x_A = b for every unit vector b (linearity)
  for (uint32_t k = 0; k < A.size(); ++k) {
    std::vector<uint32_t> u(bw, 0);
    u[A[k] >> 5] = 1u << (A[k] & 31);
    transform_words(u, N);
    for (uint32_t w = 0; w < bw; ++w) u[w] &= info[w];
    transform_words(u, N);
    for (uint32_t w = 0; w < bw; ++w) {
      uint32_t want = (w == (A[k] >> 5)) ? (1u << (A[k] & 31)) : 0u;
      if ((u[w] & info[w]) != want) return POLAR_ENOTSYS;
    }
  }

  // ---- pruned tree -> node program (Sec. II-B3; precedence R0, R1, REP, SPC)
  hp.prog.clear();
  hp.counts = {};
  auto fits = [](uint32_t lim, uint32_t m) { return lim == 0 || m <= lim; };
  auto nfrozen = [&](uint32_t s, uint32_t m) {
    uint32_t c = 0;
    for (uint32_t j = s; j < s + m; ++j) c += bit(frozen, j) ? 1 : 0;
    return c;
  };
  struct Emit {
    static void go(HostPlan& hp, const polar_plan_desc& d, const std::vector<uint32_t>& fz,
                   uint32_t s, uint32_t m, uint32_t dep,
                   const decltype(fits)& fits, const decltype(nfrozen)& nfrozen) {
      if (m == 1) {
        bool f = (fz[s >> 5] >> (s & 31)) & 1u;
        hp.prog.push_back(op_make(f ? OP_LF : OP_LI, dep, s));
        (f ? hp.counts.leaf_f : hp.counts.leaf_i)++;
        return;
      }
      const uint32_t nf = nfrozen(s, m);
      const bool last_info = !((fz[(s + m - 1) >> 5] >> ((s + m - 1) & 31)) & 1u);
      const bool first_frozen = (fz[s >> 5] >> (s & 31)) & 1u;
      const uint32_t en = d.node_enable;
      uint32_t op = 0xFF;
      if ((en & POLAR_NODE_R0) && nf == m && fits(d.r0_max, m)) {
        op = OP_R0;
        hp.counts.r0++;
      } else if ((en & POLAR_NODE_R1) && nf == 0 && fits(d.r1_max, m)) {
        op = OP_R1;
        hp.counts.r1++;
      } else if ((en & POLAR_NODE_REP) && nf == m - 1 && last_info && fits(d.rep_max, m)) {
        op = OP_REP;
        hp.counts.rep++;
      } else if ((en & POLAR_NODE_SPC) && m >= 4 && nf == 1 && first_frozen && fits(d.spc_max, m)) {
        op = OP_SPC;
        hp.counts.spc++;
      }
      if (op != 0xFF) {
        hp.prog.push_back(op_make(op, dep, s));
        return;
      }
      hp.prog.push_back(op_make(OP_F, dep, s));
      go(hp, d, fz, s, m / 2, dep + 1, fits, nfrozen);
      hp.prog.push_back(op_make(OP_G, dep, s));
      go(hp, d, fz, s + m / 2, m / 2, dep + 1, fits, nfrozen);
      hp.prog.push_back(op_make(OP_H, dep, s));
    }
  };
  Emit::go(hp, d, frozen, 0, N, 0, fits, nfrozen);

  // ---- the same walk with fused steps for the single-path tier: f followed
  // by its left child, or g followed by its right child and the parent's h,
  // when that child is a dedicated node or leaf of at most 64 positions
  hp.sc_prog.clear();
  for (size_t i = 0; i < hp.prog.size(); ++i) {
    const uint32_t w = hp.prog[i], op = op_code(w), dep = op_depth(w);
    if ((op == OP_F || op == OP_G) && i + 1 < hp.prog.size() && (N >> (dep + 1)) <= 64) {
      const uint32_t nx = hp.prog[i + 1], nop = op_code(nx);
      if (nop >= OP_R0 && nop <= OP_LI && op_depth(nx) == dep + 1) {
        if (op == OP_F) {
          hp.sc_prog.push_back(op_make(OP_FN, dep, op_off(w)) | (nop << 24));
          i += 1;
          continue;
        }
        if (i + 2 < hp.prog.size() && op_code(hp.prog[i + 2]) == OP_H &&
            op_depth(hp.prog[i + 2]) == dep) {
          hp.sc_prog.push_back(op_make(OP_GNH, dep, op_off(w)) | (nop << 24));
          i += 2;
          continue;
        }
      }
    }
    hp.sc_prog.push_back(w);
  }
  // ---- and with an f-and-left-child step merged into the g, right-child and
  // h step of the same node that follows it (the register stages' program)
  hp.q_prog.clear();
  for (size_t i = 0; i < hp.sc_prog.size(); ++i) {
    const uint32_t w = hp.sc_prog[i];
    if (op_code(w) == OP_FN && i + 1 < hp.sc_prog.size()) {
      const uint32_t nx = hp.sc_prog[i + 1];
      if (op_code(nx) == OP_GNH && op_depth(nx) == op_depth(w)) {
        hp.q_prog.push_back(op_make(OP_PAIR, op_depth(w), (op_sub(w) << 8) | (op_sub(nx) << 12)));
        i += 1;
        continue;
      }
    }
    hp.q_prog.push_back(w);
  }

  // ---- CRC syndrome columns.  CRC(data) is the remainder of data(x) x^c
  // by g(x) (MSB first, init 0, no final xor), linear in the data bits: data
  // bit t contributes x^(k_data - 1 - t + c) mod g; a CRC bit contributes its
  // own unit.  A path passes iff the XOR of the columns of its 1 bits is 0.
  const uint32_t c = d.crc_len, kd = d.K - c;
  const uint32_t cmask = c == 32 ? ~0u : ((1u << c) - 1u);
  const uint32_t poly = uint32_t(d.crc_poly) & cmask;
  std::vector<uint32_t> crccol(N, 0);
  if (c > 0) {
    uint32_t r = poly;  // x^c mod g
    for (int t = int(kd) - 1; t >= 0; --t) {
      crccol[A[t]] = r;
      const bool top = (r >> (c - 1)) & 1u;
      r = (r << 1) & cmask;
      if (top) r ^= poly;
    }
    for (uint32_t t = 0; t < c; ++t) crccol[A[kd + t]] = 1u << (c - 1 - t);
  }
  std::vector<uint32_t> datamask(bw, 0), prefix(bw, 0);
  for (uint32_t t = 0; t < kd; ++t) datamask[A[t] >> 5] |= 1u << (A[t] & 31);
  for (uint32_t w = 1; w < bw; ++w) prefix[w] = prefix[w - 1] + __builtin_popcount(datamask[w - 1]);
  std::vector<uint32_t> datacomp(size_t(bw) * 8, 0);
  for (uint32_t w = 0; w < bw; ++w) {
    uint32_t* e = &datacomp[size_t(w) * 8];
    e[0] = datamask[w];
    compress_masks(datamask[w], e + 1);
    e[6] = prefix[w];
    e[7] = uint32_t(__builtin_popcount(datamask[w]));
  }

  // ---- header + blob
  const uint32_t E = elem_bytes(d.quant), KB = key_bytes(d.quant);
  // the largest layout among the schedule's stages (layouts are not monotone
  // in L: small lists keep their top buffers in global memory)
  LdsLayout lay = lds_layout(N, n, E, first, KB);
  for (uint32_t L = first; L < maxl;) {
    L = stage_after(d.algo == POLAR_PA_SCL, maxl, L);
    const LdsLayout l2 = lds_layout(N, n, E, L, KB);
    if (l2.total > lay.total) lay = l2;
  }
  if (lay.total > kLdsBudget) return POLAR_EUNSUP;  // lds_layout spills what it can

  DevPlan h{};
  h.N = N;
  h.n = n;
  h.K = d.K;
  h.c = c;
  h.n_tx = N - S - Pn;
  h.n_punct = Pn;
  h.k_data = kd;
  h.quant = d.quant;
  h.algo = d.algo;
  h.L = d.algo == POLAR_CA_SCL ? d.L : 1;
  h.L_max = maxl;
  h.n_ops = uint32_t(hp.prog.size());
  h.bw = bw;
  h.info_words = (kd + 31) / 32;
  h.code_words = (N + 31) / 32;
  h.max_list = maxl;
  h.lds_max = lay.total;
  h.first_stage = first;
  uint32_t off = sizeof(DevPlan) / 4;
  h.off_prog = off;
  off += h.n_ops;
  h.n_sc_ops = uint32_t(hp.sc_prog.size());
  h.off_sc_prog = off;
  off += h.n_sc_ops;
  h.n_q_ops = uint32_t(hp.q_prog.size());
  h.off_q_prog = off;
  off += h.n_q_ops;
  h.off_infomask = off;
  off += bw;
  h.off_datamask = off;
  off += bw;
  h.off_dataprefix = off;
  off += bw;
  off = (off + 3u) & ~3u;  // 16-byte entries, read as two 16-byte loads
  h.off_datacomp = off;
  off += bw * 8;
  h.off_crccol = off;
  off += N;
  h.off_crcpos = off;
  off += std::max(c, 1u);
  const uint32_t nnib = (N + 3) / 4;
  h.off_crcnib = off;
  off += nnib * 16;
  hp.blob.assign(off, 0);
  std::copy_n(reinterpret_cast<const uint32_t*>(&h), sizeof(DevPlan) / 4, hp.blob.begin());
  std::copy(hp.prog.begin(), hp.prog.end(), hp.blob.begin() + h.off_prog);
  std::copy(hp.sc_prog.begin(), hp.sc_prog.end(), hp.blob.begin() + h.off_sc_prog);
  std::copy(hp.q_prog.begin(), hp.q_prog.end(), hp.blob.begin() + h.off_q_prog);
  std::copy(info.begin(), info.end(), hp.blob.begin() + h.off_infomask);
  std::copy(datamask.begin(), datamask.end(), hp.blob.begin() + h.off_datamask);
  std::copy(prefix.begin(), prefix.end(), hp.blob.begin() + h.off_dataprefix);
  std::copy(datacomp.begin(), datacomp.end(), hp.blob.begin() + h.off_datacomp);
  std::copy(crccol.begin(), crccol.end(), hp.blob.begin() + h.off_crccol);
  for (uint32_t t = 0; t < c; ++t) hp.blob[h.off_crcpos + t] = A[kd + t];
  // nibble table of the syndrome columns (Sec. IV-B: a table of
  // precomputed sub-results lets the CRC advance several bits per lookup)
  for (uint32_t q = 0; q < nnib; ++q)
    for (uint32_t e = 0; e < 16; ++e) {
      uint32_t v = 0;
      for (uint32_t b = 0; b < 4; ++b)
        if (((e >> b) & 1u) && 4 * q + b < N) v ^= crccol[4 * q + b];
      hp.blob[h.off_crcnib + q * 16 + e] = v;
    }
  hp.hdr = h;
  hp.frozen = frozen;
  hp.desc = d;
  hp.desc.frozen = nullptr;
  return POLAR_OK;
}

uint64_t stage_work(const HostPlan& hp, uint32_t L) {
  const uint32_t N = hp.hdr.N;
  uint64_t ops = 0, a = 1;
  auto clog2 = [](uint64_t x) {
    uint64_t k = 0;
    while ((1ull << k) < x) ++k;
    return k;
  };
  for (uint32_t w : hp.prog) {
    const uint32_t op = op_code(w), m = N >> op_depth(w);
    uint64_t C = 1;
    switch (op) {
      case OP_F:
      case OP_G:
      case OP_H: ops += a * (m / 2); continue;
      case OP_R0:
      case OP_LF: C = 1; break;
      case OP_LI:
      case OP_REP: C = 2; break;
      case OP_R1: C = 4; break;
      default: C = 8; break;
    }
    ops += a * m;
    if (C > 1) {
      const uint64_t tot = a * C;
      ops += tot * clog2(tot);
      a = std::min<uint64_t>(L, tot);
    }
  }
  ops += a * hp.hdr.K + a * clog2(a);
  return ops;
}

uint32_t plan_lds_bytes(const DevPlan& h, uint32_t L) {
  return lds_layout(h.N, h.n, elem_bytes(h.quant), L, key_bytes(h.quant)).total;
}

}  // namespace polar
