"""Mutation check of the oracle's pins (CPU only; not collected by pytest).

Each entry below plants one plausible mistake in a copy of oracle/oracle.cpp
(a dropped clamp, a wrong sign, a swapped tie-break, ...).  For each one the
script builds the modified copy into a temporary directory, points the
oracle binding at it (POLAR_ORACLE_LIB_OVERRIDE) and runs the pin tests.  A
mutation is "caught" when at least one pin fails.  The repository's own
oracle is never modified.

    python tests/oracle_mutations.py            # every mutation
    python tests/oracle_mutations.py key_order  # selected ones

Exit status 0 when every mutation is caught.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.cpp")
PIN_TESTS = ["tests/test_oracle_pins.py", "tests/test_oracle_hand.py"]

# name -> (text to replace, replacement); the text must occur exactly once
MUTATIONS = {
    # Sec. III-B3: the integer path metric saturates at Q
    "pm_no_clamp": ("static P pm_add(P pm, Acc pen) { return std::min<int64_t>((int64_t)pm + pen, Q); }",
                    "static P pm_add(P pm, Acc pen) { return (P)((int64_t)pm + pen); }"),
    # Sec. III-B3: g saturates
    "g_no_sat": ("return sat(s ? ((int32_t)b - (int32_t)a) : ((int32_t)b + (int32_t)a));",
                 "return (V)(s ? ((int32_t)b - (int32_t)a) : ((int32_t)b + (int32_t)a));"),
    # near-tie flag (float modes): always set
    "tie_always": ("bool near_tie() const { return near_tie_; }",
                   "bool near_tie() const { return true; }"),
    # near-tie flag: never set at a selection boundary
    "tie_no_boundary": ("if (hi - lo <= 1e-4 * std::max(1.0, std::fabs(lo))) near_tie_ = true;",
                        "if (hi - lo <= 1e-4 * std::max(1.0, std::fabs(lo))) (void)0;"),
    # near-tie flag: never set at the final CRC choice
    "tie_no_crc_choice": (
        "if (d <= 1e-4 * std::max(1.0, std::fabs(A::as_double(pm_[chosen])))) near_tie_ = true;",
        "if (d <= 1e-4 * std::max(1.0, std::fabs(A::as_double(pm_[chosen])))) (void)0;"),
    # near-tie flag: only the last stage's
    "tie_last_stage_only": ("tie = tie || dec.near_tie();", "tie = dec.near_tie();"),
    # selection key (metric, local index, parent) instead of (metric, parent, local index)
    "key_order": ("      if (x.parent != y.parent) return x.parent < y.parent;\n      return x.local < y.local;",
                  "      if (x.local != y.local) return x.local < y.local;\n      return x.parent < y.parent;"),
    # hard decision of 0 taken as 1 (integer modes)
    "hd_le_int": ("  static bool hd(V v) { return v < 0; }\n  static Acc mag(V v) { return std::abs((int32_t)v); }",
                  "  static bool hd(V v) { return v <= 0; }\n  static Acc mag(V v) { return std::abs((int32_t)v); }"),
    # hard decision of 0 taken as 1 (float modes)
    "hd_le_float": ("  static bool hd(V v) { return v < 0; }\n  static Acc mag(V v) { return std::fabs(v); }",
                    "  static bool hd(V v) { return v <= 0; }\n  static Acc mag(V v) { return std::fabs(v); }"),
    # f: wrong sign rule
    "f_sign": ("    V mag = std::min(std::fabs(a), std::fabs(b));\n    bool neg = (a < 0) != (b < 0);",
               "    V mag = std::min(std::fabs(a), std::fabs(b));\n    bool neg = (a < 0) && (b < 0);"),
    # g: partial sum applied with the wrong sign
    "g_sign": ("static V g(V a, V b, int s) { return s ? (b - a) : (b + a); }",
               "static V g(V a, V b, int s) { return s ? (b + a) : (b - a); }"),
    # h: left partial sums not combined with the right ones
    "h_no_xor": ("s_[p][os + i] = s_[p][os + i] ^ s_[p][os + h + i];",
                 "s_[p][os + i] = s_[p][os + h + i];"),
    # Chase / SPC positions: most reliable instead of least reliable
    "chase_largest": ("          if (mx != my) return mx < my;", "          if (mx != my) return mx > my;"),
    # SPC: candidates of the wrong parity
    "spc_parity": ("(__builtin_popcount(mask) & 1) != parity", "(__builtin_popcount(mask) & 1) == parity"),
    # SPC: three flip positions instead of four
    "spc_three": ("const int T = (kind == K_R1) ? 2 : std::min(m, 4);",
                  "const int T = (kind == K_R1) ? 2 : std::min(m, 3);"),
    # REP: candidate penalties swapped
    "rep_swap": ("Cand cd{A::pm_add(pm_[p], disagree_sum(al, m, v)), p, v,",
                 "Cand cd{A::pm_add(pm_[p], disagree_sum(al, m, 1 - v)), p, v,"),
    # integer metrics never normalised
    "no_normalise": ("if (!A::kInt || a_ == 0) return;", "return;"),
    # float penalty sums in sequential order instead of stride halving
    "sum_sequential": ("  if (m == 0) return Acc(0);\n  for (size_t s",
                       "  if (m == 0) return Acc(0);\n  { Acc t = v[0]; for (size_t i = 1; i < m; ++i) t = t + v[i]; return t; }\n  for (size_t s"),
    # CRC register initialised to ones
    "crc_init_ones": ("  uint64_t reg = 0;\n  for (int i = 0; i < nbits; ++i) {",
                      "  uint64_t reg = mask;\n  for (int i = 0; i < nbits; ++i) {"),
    # final selection ignores the CRC
    "select_ignores_crc": ("if (cl == 0 || crc_bits(b.data(), K - cl, cl, c_.crc_poly) == tail_value(b)) {",
                           "if (true) {"),
    # FA schedule skips list sizes
    "fa_quadruple": ("        st.push_back(l);\n        l *= 2;", "        st.push_back(l);\n        l *= 4;"),
    # Bhattacharyya recursion with the children swapped
    "bhatt_swap": ("      if ((i >> b) & 1)\n        lz = 2.0 * lz;", "      if (!((i >> b) & 1))\n        lz = 2.0 * lz;"),
    # reliability ties broken towards the smaller index
    "rank_tie_low": ("    if (lz[a] != lz[b]) return lz[a] < lz[b];\n    return a > b;",
                     "    if (lz[a] != lz[b]) return lz[a] < lz[b];\n    return a < b;"),
    # design rate counts the CRC bits as information
    "rate_with_crc": ("const double rate = (double)(K - crc_len) / (double)(N - S - P);",
                      "const double rate = (double)K / (double)(N - S - P);"),
    # shortened positions given the most unreliable value
    "known_neg": ("  static V known() { return (V)Q; }", "  static V known() { return (V)-Q; }"),
    # punctured positions given a certain-zero value
    "punct_known": ("for (int i = 0; i < P; ++i) chan[i] = V(0);",
                    "for (int i = 0; i < P; ++i) chan[i] = A::known();"),
    # quantiser truncates instead of rounding
    "quant_trunc": ("double q = std::nearbyint(llr[i] * scale);", "double q = std::trunc(llr[i] * scale);"),
}


def run(names):
    src = open(SRC).read()
    results = {}
    with tempfile.TemporaryDirectory() as tmp:
        for name in names:
            old, new = MUTATIONS[name]
            if src.count(old) != 1:
                results[name] = f"pattern found {src.count(old)} times"
                continue
            path = os.path.join(tmp, f"{name}.cpp")
            lib = os.path.join(tmp, f"lib{name}.so")
            with open(path, "w") as f:
                f.write(src.replace(old, new))
            subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                                   "-fPIC", "-shared", "-pthread", "-o", lib, path])
            env = dict(os.environ, POLAR_ORACLE_LIB_OVERRIDE=lib)
            r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                                "-p", "no:cacheprovider", *PIN_TESTS],
                               cwd=ROOT, env=env, capture_output=True, text=True)
            failed = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
            results[name] = ("caught: " + failed[0][7:]) if r.returncode else "NOT CAUGHT"
            print(f"{name:22s} {results[name]}", flush=True)
    return results


if __name__ == "__main__":
    names = sys.argv[1:] or list(MUTATIONS)
    res = run(names)
    missed = [n for n, v in res.items() if not v.startswith("caught")]
    print(f"{len(res) - len(missed)} of {len(res)} mutations caught" +
          (f"; not caught: {', '.join(missed)}" if missed else ""))
    sys.exit(1 if missed else 0)
