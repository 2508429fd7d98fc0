"""CPU-only checks of the C-ABI library: it loads, exports every function
that include/polar_scl.h declares, and its host planner agrees with the
oracle's construction and tree decomposition (no device is touched)."""
import collections
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1710_08314_amd import polar as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "polar_scl.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(polar_\w+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(P.LIB_PATH)
    names = header_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(P.EXPORTS)


def test_strerror_and_version():
    assert P.lib.polar_strerror(0) == b"success"
    assert P.lib.polar_strerror(-5).startswith(b"frozen set")
    assert P.lib.polar_version().startswith(b"polar-scl")


CONFIGS = [  # (N, K, c, design, S, rep_max)
    (256, 128, 8, 2.0, 0, 0), (2048, 1723, 32, 4.5, 0, 8), (1024, 512, 24, 2.5, 0, 0),
    (512, 200, 11, 2.5, 60, 0), (128, 40, 11, 1.5, 0, 0), (32, 12, 11, 1.5, 0, 8),
    (2, 1, 0, 0.0, 0, 0), (8, 4, 0, 1.0, 0, 0), (2048, 300, 11, 2.5, 512, 0),
]


@pytest.mark.parametrize("N,K,c,design,S,rep_max", CONFIGS)
def test_frozen_set_matches_oracle_construction(N, K, c, design, S, rep_max):
    info, fz = P.plan_query(N, K, c, 0x621, design_ebn0_db=design, n_shorten=S, rep_max=rep_max)
    assert np.array_equal(fz, O.construct(N, K, S, c, design))
    assert info.n_tx == N - S and info.k_data == K - c
    assert info.info_words == (K - c + 31) // 32


@pytest.mark.parametrize("N,K,c,design,S,rep_max", CONFIGS)
@pytest.mark.parametrize("spc_max", [4, 0])
def test_node_program_matches_oracle_tree(N, K, c, design, S, rep_max, spc_max):
    info, fz = P.plan_query(N, K, c, 0x621, design_ebn0_db=design, n_shorten=S, rep_max=rep_max,
                            spc_max=spc_max)
    code = O.Code(N, K, fz, c, 0x621, S=S, rep_max=rep_max, spc_max=spc_max)
    cnt = collections.Counter(k for k, _, _ in O.nodes(code))
    assert (info.n_r0, info.n_r1, info.n_rep, info.n_spc, info.n_leaf_frozen,
            info.n_leaf_info) == (cnt["R0"], cnt["R1"], cnt["REP"], cnt["SPC"], cnt["LEAF_F"],
                                  cnt["LEAF_I"])
    # F, G, H for every split node + one op per leaf-level node
    n_nodes = sum(cnt.values())
    assert info.n_ops == n_nodes + 3 * (n_nodes - 1)


def test_headline_code_tree():
    # the (2048, 1723 incl. CRC-32) code of the paper's Table III / Table IV
    info, _ = P.plan_query(2048, 1723, 32, 0x04C11DB7, design_ebn0_db=4.5, algo=P.FA_SCL,
                           L_max=32, quant=P.I8)
    assert (info.n_r0, info.n_rep, info.n_r1, info.n_spc) == (19, 20, 71, 29)
    assert info.max_list == 32
    assert info.lds_bytes <= 160 * 1024


def test_explicit_frozen_mask_roundtrip():
    rng = np.random.default_rng(0)
    fz = np.ones(64, np.uint8)
    fz[[63, 62, 61, 59, 55, 47, 31, 60]] = 0
    info, back = P.plan_query(64, 8, 0, 0, frozen=fz)
    assert np.array_equal(back, fz)


@pytest.mark.parametrize("kw,code", [
    (dict(N=100, K=10), -1), (dict(N=4096, K=10), -2), (dict(N=64, K=0), -1),
    (dict(N=64, K=65), -1), (dict(N=64, K=10, n_shorten=60), -1),
    (dict(N=64, K=10, crc_len=10), -1), (dict(N=64, K=40, crc_len=33), -2),
    (dict(N=64, K=10, algo=P.CA_SCL, L=3), -1), (dict(N=64, K=10, algo=P.CA_SCL, L=64), -2),
    (dict(N=64, K=10, algo=P.FA_SCL, L_max=8), -1),  # FA without a CRC
    (dict(N=64, K=10, quant=7), -1),
    (dict(N=64, K=10, n_puncture=64), -1), (dict(N=64, K=10, n_shorten=20, n_puncture=44), -1),
    (dict(N=64, K=30, n_shorten=20, n_puncture=20), -1),  # K > N - S - P
])
def test_plan_errors(kw, code):
    with pytest.raises(P.PolarError) as e:
        P.plan_query(**kw)
    assert e.value.code == code


def test_systematic_check_agrees_with_oracle_encoder():
    # the plan rejects (-5) exactly the information sets for which the
    # two-pass encoder of Sec. II-A does not give x_A = b
    import itertools
    N = 8
    n_bad = 0
    for K in (2, 3, 4):
        for A in itertools.combinations(range(N), K):
            fz = np.ones(N, np.uint8)
            fz[list(A)] = 0
            eye = np.eye(K, dtype=np.uint8)
            ok = all((O.encode(fz, eye[k])[list(A)] == eye[k]).all() for k in range(K))
            if ok:
                P.plan_query(N, K, frozen=fz)
            else:
                n_bad += 1
                with pytest.raises(P.PolarError) as e:
                    P.plan_query(N, K, frozen=fz)
                assert e.value.code == -5
    assert n_bad > 10


def test_given_mask_must_freeze_shortened_positions():
    fz = np.ones(32, np.uint8)
    fz[[31, 30, 29, 27]] = 0
    with pytest.raises(P.PolarError):
        P.plan_query(32, 4, frozen=fz, n_shorten=2)


@pytest.mark.parametrize("N,K,c,design,S,Pn", [
    (256, 90, 11, 1.5, 0, 37), (512, 192, 0, 3.0, 0, 192), (1024, 400, 24, 2.5, 100, 150),
    (2048, 1000, 11, 2.5, 256, 300), (64, 20, 11, 1.0, 5, 9),
])
def test_punctured_frozen_set_matches_oracle(N, K, c, design, S, Pn):
    """Puncturing: the plan's construction equals the oracle's, the sent
    length is N - S - P, and a given frozen set must freeze [0, P)."""
    info, fz = P.plan_query(N, K, c, 0x621, design_ebn0_db=design, n_shorten=S, n_puncture=Pn)
    assert np.array_equal(fz, O.construct(N, K, S, c, design, P=Pn))
    assert info.n_tx == N - S - Pn
    bad = fz.copy()
    j = int(np.where(fz[Pn:] == 0)[0][0]) + Pn
    bad[j], bad[Pn - 1] = 1, 0  # an information bit inside the punctured head
    with pytest.raises(P.PolarError):
        P.plan_query(N, K, c, 0x621, frozen=bad, n_shorten=S, n_puncture=Pn)


def test_spilled_layouts_of_n2048():
    """Which LLR buffers of an N = 2048 frame live in global memory instead of
    LDS: for lists of at most 4 the root (N elements) and the slots of depths
    1 and 2 (L x (1024 + 512)); for L = 8 none; for L >= 16 the slots of the
    top depths, one to three of them (L x 1024 at least, L x (1024 + 512 +
    256) at most), so that float32 at L = 32 (272 KB otherwise) fits one
    CU's LDS and int8 at L = 32 fits 32 KB.  The LDS figure of a plan is that
    of its largest stage."""
    E = {P.F32: 4, P.I16: 2, P.I8: 1}
    for q in (P.F32, P.I16, P.I8):
        for L in (1, 2, 4, 8, 16, 32):
            info, _ = P.plan_query(2048, 1000, 11, 0x621, design_ebn0_db=2.5, algo=P.CA_SCL,
                                   L=L, quant=q)
            full = E[q] * (2048 + L * 2047)  # root + the slots of depths 1..11
            assert info.lds_bytes <= 160 * 1024 - 1024
            if L <= 4:
                small = full - E[q] * (2048 + L * (1024 + 512))
                assert small <= info.lds_bytes < small + 8 * 1024, (q, L)
            elif L == 8:
                assert info.lds_bytes >= full
            else:
                most = full - E[q] * L * (1024 + 512 + 256)
                least = full - E[q] * L * 1024
                assert most <= info.lds_bytes < least + 16 * 1024, (q, L)
    i8, _ = P.plan_query(2048, 1000, 11, 0x621, design_ebn0_db=2.5, algo=P.CA_SCL, L=32,
                         quant=P.I8)
    assert i8.lds_bytes <= 32 * 1024
    # a fully adaptive plan reports its largest stage (L = 8 here, all in LDS)
    fa, _ = P.plan_query(2048, 1000, 11, 0x621, design_ebn0_db=2.5, algo=P.FA_SCL, L_max=8,
                         quant=P.I8)
    assert fa.lds_bytes >= 2048 + 8 * 2047
    # codes shorter than 1024 keep everything in LDS at small lists
    sm, _ = P.plan_query(512, 256, 11, 0x621, design_ebn0_db=2.5, algo=P.CA_SCL, L=4,
                         quant=P.I8)
    assert sm.lds_bytes >= 512 + 4 * 511
