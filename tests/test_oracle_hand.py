"""Hand-derived decodes that pin the oracle's selection rules (CPU only).

Each case is small enough to follow on paper, and its expected outputs are
written out from the method, not taken from the oracle.  The derivation of
every value sits beside it.  The cases pin what brute force and closed forms
leave open: the saturation of integer path metrics, the selection key's
tie-break order, the near-tie flag of the float modes, and the order of float
penalty sums.

Notation (Sec. II-B1): f(a, b) = sign(a) sign(b) min(|a|, |b|), g(a, b, s) =
b + (1 - 2 s) a, HD(v) = [v < 0].  For N = 4, the decoder splits the root
LLRs (l0, l1, l2, l3) into the left child (f(l0, l2), f(l1, l3)) and, after
the left half is decided with partial sums (s0, s1), the right child
(g(l0, l2, s0), g(l1, l3, s1)).  A size-2 node (a, b) gives u_left the LLR
f(a, b) and u_right the LLR g(a, b, u_left).  The codeword estimate is
x = (u0^u1^u2^u3, u1^u3, u2^u3, u3); with every position in A (no frozen
bit), the systematic information vector is b = x.

The test CRC is c = 2 with g(x) = x^2 + x + 1 (poly 0b11): long division of
d(x) x^2 gives CRC(00) = 00, CRC(01) = 11, CRC(10) = 01, CRC(11) = 10, so the
valid 4-bit vectors (data, CRC) are 0000, 0111, 1001 and 1110.
"""
import numpy as np
import pytest

import oracle as O

ALL_INFO = np.zeros(4, dtype=np.uint8)
CRC2 = (2, 0b11)


def test_crc2_table():
    # the four valid words quoted in the module docstring
    for data, crc in [((0, 0), 0b00), ((0, 1), 0b11), ((1, 0), 0b01), ((1, 1), 0b10)]:
        assert O.crc(np.array(data, np.uint8), *CRC2) == crc


@pytest.mark.parametrize("quant,Q,llr,pens", [
    # int8: |l| = (100, 100, 60, 100); pens of the four Chase masks 0, 60, 100, 60+100
    (O.I8, 127, [-100, 100, 60, 100], [0, 60, 100, 160]),
    # int16: |l| = (30000, 30000, 20000, 30000)
    (O.I16, 32767, [-30000, 30000, 20000, 30000], [0, 20000, 30000, 50000]),
])
def test_int_path_metric_saturates_at_Q(quant, Q, llr, pens):
    """Sec. III-B3: the integer path metric saturates after every update.

    All four positions are information, so the root is one Rate-1 node of
    size 4 (Sec. II-B3).  HD(l) = (1, 0, 0, 0).  Chase-2 flips the two least
    reliable positions, ordered by (|l|, index): position 2 (|l| = 60), then
    position 0 (100, the smallest index among the ties).  The masks give the
    penalties 0, |l2|, |l0|, |l2| + |l0|; the last exceeds Q, and the sum,
    exact in int32, saturates once when added to the metric 0.  L = 4 keeps
    every candidate.  The output is the hard decision with metric 0."""
    code = O.Code(4, 4, ALL_INFO, 0, 0, quant=quant, algo=O.CA_SCL, L=4)
    r = O.decode(code, np.array([llr], dtype=O.DTYPES[quant]))
    expect = [min(p, Q) for p in pens]
    assert r.pm_list[0].tolist() == expect
    assert r.pm_list[0][3] == Q and pens[3] > Q
    assert r.info[0].tolist() == [1, 0, 0, 0]
    assert r.n_pm[0] == 4 and r.pm[0] == 0


def test_selection_key_is_metric_parent_local():
    """Sec. II-B2 selection with the key (metric, parent rank, local index).

    int8, leaves only, L = 2, channel LLRs (0, 0, -64, -64).
      * Left child: (f(0, -64), f(0, -64)) = (0, 0).  u0: LLR f(0, 0) = 0;
        both bits cost 0; keys (0, p0, 0), (0, p0, 1); ranks r0: u0 = 0,
        r1: u0 = 1.
      * u1: LLR g(0, 0, u0) = 0 on both paths; four keys of metric 0.  The
        key order (metric, parent, local) keeps (0, r0, 0) and (0, r0, 1):
        u = (0, 0) and (0, 1).  (Ordered by (metric, local, parent) it would
        keep (0, 0) and (1, 0).)
      * Right child: g(0, -64, s0) = g(0, -64, s1) = -64 on both paths.
        u2: LLR f(-64, -64) = 64, so bit 0 costs 0 and bit 1 costs 64: each
        path takes 0, ranks kept.  u3: LLR g(-64, -64, 0) = -128, saturated
        to -127: bit 1 costs 0; each path takes 1.
      * Survivors: r0 u = (0, 0, 0, 1), x = 1111; r1 u = (0, 1, 0, 1),
        x = 0011.  Neither is a valid CRC word (1111: CRC(11) = 10; 0011:
        CRC(00) = 00), so the output is rank 0 with crc_ok = 0: data (1, 1).
        Under the wrong order r1 would be u = (1, 0, 0, 1), x = 0111, which
        passes.  Every metric is 0 after normalisation."""
    code = O.Code(4, 4, ALL_INFO, *CRC2, quant=O.I8, algo=O.CA_SCL, L=2, node_enable=0)
    r = O.decode(code, np.array([[0, 0, -64, -64]], dtype=np.int8))
    assert r.crc_ok[0] == 0
    assert r.info[0].tolist() == [1, 1]
    assert r.xhat[0].tolist() == [1, 1, 1, 1]
    assert r.pm_list[0].tolist() == [0, 0]
    assert r.L_used[0] == 2 and r.n_pm[0] == 2


def test_near_tie_at_the_selection_boundary():
    """R-21: a frame is flagged when the L-th and (L+1)-th keys of a
    selection are within 1e-4 relative.

    float32, Rate-1 root of size 4, L = 2, LLRs (-1, 1, 1, 1): HD = (1, 0,
    0, 0); all |l| = 1, so Chase-2 flips positions 0 and 1 (index order).
    Candidate metrics 0, 1, 1, 2; the second and third are equal, so the
    boundary of the L = 2 selection is a tie.  The final choice (no CRC) is
    rank 0 at metric 0 against rank 1 at 1: a clear gap.  Output: HD."""
    code = O.Code(4, 4, ALL_INFO, 0, 0, quant=O.F32, algo=O.CA_SCL, L=2)
    r = O.decode(code, np.array([[-1.0, 1.0, 1.0, 1.0]], dtype=np.float32))
    assert r.near_tie[0] == 1
    assert r.pm_list[0].tolist() == [0.0, 1.0]
    assert r.info[0].tolist() == [1, 0, 0, 0]


def test_no_near_tie_with_a_clear_gap():
    """LLRs (-1, 1.001, 1.5, 1.5) (float32): Chase-2 flips position 0 (|l| =
    1) and position 1 (1.001).  Metrics 0, 1, 1.001, 2.001: the boundary of
    the L = 2 selection is 1 against 1.001, a gap of 1e-3 > 1e-4 max(1, 1).
    The final choice: 0 against 1.  Not flagged."""
    code = O.Code(4, 4, ALL_INFO, 0, 0, quant=O.F32, algo=O.CA_SCL, L=2)
    llr = np.array([[-1.0, 1.001, 1.5, 1.5]], dtype=np.float32)
    r = O.decode(code, llr)
    assert r.near_tie[0] == 0
    assert r.pm_list[0][0] == 0.0 and r.pm_list[0][1] == 1.0
    # the same frame at L = 1: the Rate-1 decision's margin is |l0| = 1
    r1 = O.decode(O.Code(4, 4, ALL_INFO, 0, 0, quant=O.F32, algo=O.SC), llr)
    assert r1.near_tie[0] == 0


def test_near_tie_at_the_final_choice():
    """R-21: the final choice is a near-tie when another path that passes
    the CRC (here every path: no CRC) has the chosen metric within 1e-4.

    LLRs (0, 1, 1, 1), float32, Rate-1 root, L = 4: HD = (0, 0, 0, 0); the
    least reliable positions are 0 (|l| = 0) and 1.  Candidate metrics 0, 0,
    1, 1: L = 4 keeps all four, so no selection has a boundary; ranks 0 and
    1 both have metric 0, and the output (rank 0, the hard decision) is a
    near-tie."""
    code = O.Code(4, 4, ALL_INFO, 0, 0, quant=O.F32, algo=O.CA_SCL, L=4)
    r = O.decode(code, np.array([[0.0, 1.0, 1.0, 1.0]], dtype=np.float32))
    assert r.near_tie[0] == 1
    assert r.pm_list[0].tolist() == [0.0, 0.0, 1.0, 1.0]
    assert r.info[0].tolist() == [0, 0, 0, 0]


def test_near_tie_of_an_earlier_stage_is_kept():
    """FA-SSCL (Sec. II-B5) with L = 1 then 2: a tie that only the failed
    first stage met still flags the frame.

    float32, leaves only, LLRs (0, -2, -5, -3), CRC of the module docstring.
      * Left child: (f(0, -5), f(-2, -3)) = (-0, 2).
      * Stage L = 1: u0 has LLR f(-0, 2) = 0, both bits cost 0: the L = 1
        selection keeps bit 0 over an equal key, a tie.  u1: LLR g(-0, 2, 0)
        = 2, bit 0.  Right child: (g(0, -5, 0), g(-2, -3, 0)) = (-5, -5);
        u2: LLR 5, bit 0; u3: LLR -10, bit 1.  u = (0, 0, 0, 1), x = 1111:
        CRC fails.
      * Stage L = 2: u0 forks into two paths of metric 0 (two candidates,
        both kept: no boundary).  u1: LLR 2 on both; keys 0, 0, 2, 2; the
        boundary is 0 against 2.  Both paths see the right child (-5, -5)
        and take u2 = 0 (boundary 0 against 5) and u3 = 1 (0 against 10).
        Rank 0: u = (0, 0, 0, 1), x = 1111, fails.  Rank 1: u = (1, 0, 0, 1),
        x = 0111, passes: the output, data (0, 1), and no other passing path
        to tie with.
    Only stage 1 met a tie, and the flag covers the whole decode."""
    code = O.Code(4, 4, ALL_INFO, *CRC2, quant=O.F32, algo=O.FA_SCL, L_max=2, node_enable=0)
    r = O.decode(code, np.array([[0.0, -2.0, -5.0, -3.0]], dtype=np.float32))
    assert r.L_used[0] == 2 and r.crc_ok[0] == 1
    assert r.info[0].tolist() == [0, 1]
    assert r.xhat[0].tolist() == [0, 1, 1, 1]
    assert r.near_tie[0] == 1
    # the second stage alone (CA-SCL L = 2) meets no tie
    ca = O.decode(O.Code(4, 4, ALL_INFO, *CRC2, quant=O.F32, algo=O.CA_SCL, L=2, node_enable=0),
                  np.array([[0.0, -2.0, -5.0, -3.0]], dtype=np.float32))
    assert ca.near_tie[0] == 0 and ca.info[0].tolist() == [0, 1]


def test_int_modes_never_flag_near_ties():
    # the flag is defined for the float modes only (integer decoding is exact)
    code = O.Code(4, 4, ALL_INFO, 0, 0, quant=O.I16, algo=O.CA_SCL, L=2)
    r = O.decode(code, np.array([[-1, 1, 1, 1]], dtype=np.int16))
    assert r.near_tie[0] == 0 and r.pm_list[0].tolist() == [0, 1]


def test_float_penalty_sum_order():
    """R-20: float penalty sums use stride halving, v[i] += v[i + s] for
    s = m/2 ... 1.

    Every position frozen: the root is one Rate-0 node of size 4, whose
    penalty is the sum of |l_i| [l_i < 0].  LLRs (-2^24, -1, -0.0, -1) give
    the terms (2^24, 1, 0, 1) (HD(-0.0) = 0: no term).  Stride halving:
    (2^24 + 0, 1 + 1) = (2^24, 2), then 2^24 + 2 = 16777218, exact in
    float32.  Summed left to right, 2^24 + 1 rounds to 2^24 (half to even)
    and the result is 16777216."""
    fz = np.ones(4, dtype=np.uint8)
    code = O.Code(4, 0, fz, 0, 0, quant=O.F32, algo=O.SC)
    r = O.decode(code, np.array([[-(2.0 ** 24), -1.0, -0.0, -1.0]], dtype=np.float32))
    assert r.pm[0] == 16777218.0
