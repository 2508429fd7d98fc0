"""Shared helpers of the GPU tests: oracle-made inputs, GPU decode, and the
element-by-element comparison against the oracle.

Inputs are always built on the host: seeded bits and noise from
paper_1710_08314_amd.synth, CRC + systematic encoding + BPSK/AWGN + LLR
quantisation by the oracle.  The GPU decoder then consumes those exact LLR
buffers; nothing the GPU produces is fed back to the oracle.
"""
from __future__ import annotations

import numpy as np

import oracle as O
from paper_1710_08314_amd import synth

QMAP = {"f32": O.F32, "i16": O.I16, "i8": O.I8}
AMAP = {"sc": O.SC, "ca": O.CA_SCL, "pa": O.PA_SCL, "fa": O.FA_SCL}

# float32 parity tolerance on path metrics: |dPM| <= 1e-4 max(1, |PM|)
PM_RTOL = 1e-4


def oracle_code(N, K, c, poly, frozen, S=0, quant="f32", algo="ca", L=1, L_max=1,
                node_enable=O.NODE_ALL, rep_max=None, spc_max=4, r1_max=0, r0_max=0):
    q = QMAP[quant] if isinstance(quant, str) else quant
    if rep_max is None:
        rep_max = 8 if q == O.I8 else 0
    return O.Code(N, K, frozen, c, poly, S=S, quant=q, algo=AMAP[algo] if isinstance(algo, str)
                  else algo, L=L, L_max=L_max, node_enable=node_enable, rep_max=rep_max,
                  spc_max=spc_max, r1_max=r1_max, r0_max=r0_max)


def make_inputs(code: O.Code, n: int, seed: int, ebn0_db: float, first: int = 0):
    """Data bits [n, K-c] and quantised LLRs [n, N-S] built by the oracle."""
    bits, noise = synth.frames(seed, first, n, code.k_data, code.n_tx)
    x = np.zeros((n, code.n_tx), dtype=np.uint8)
    for f in range(n):
        b = O.attach_crc(bits[f], code.crc_len, code.crc_poly)
        x[f] = O.encode(code.frozen, b)[:code.n_tx]
    sigma = synth.sigma_for(ebn0_db, code.k_data, code.n_tx)
    return bits, O.make_llr(code, x, noise, sigma)


def gpu_plan(code: O.Code):
    from paper_1710_08314_amd import polar as P

    return P.Plan(code.N, code.K, code.crc_len, code.crc_poly, frozen=code.frozen,
                  n_shorten=code.S, algo=code.algo, L=code.L, L_max=code.L_max, quant=code.quant,
                  node_enable=code.node_enable, rep_max=code.rep_max, spc_max=code.spc_max,
                  r1_max=code.r1_max, r0_max=code.r0_max)


def gpu_decode(code: O.Code, llr: np.ndarray, plan=None, schedule=0):
    import torch
    from paper_1710_08314_amd import polar as P

    plan = plan or gpu_plan(code)
    t = torch.from_numpy(np.ascontiguousarray(llr)).cuda()
    info, status, pml = P.decode_batch(plan, t, with_pm_lists=True, schedule=schedule)
    torch.cuda.synchronize()
    info = info.cpu().numpy().view(np.uint32)
    st = P.status_fields(status.cpu().numpy())
    pml = pml.cpu().numpy().view(np.uint32)
    bits = P.unpack_bits(info, code.k_data)
    return bits, st, pml


def pm_values(bits_u32: np.ndarray, quant) -> np.ndarray:
    if quant == O.F32:
        return bits_u32.view(np.float32).astype(np.float64)
    return bits_u32.view(np.int32).astype(np.float64)


def compare(code: O.Code, llr: np.ndarray, ref: O.Result | None = None, schedule=0):
    """Decode on both sides and assert parity.  Returns a small report."""
    ref = ref if ref is not None else O.decode(code, llr, threads=8)
    bits, st, pml = gpu_decode(code, llr, schedule=schedule)
    F = llr.shape[0]
    ml = code.max_list()
    g_pm = pm_values(st["pm_bits"], code.quant)
    g_list = np.full((F, ml), np.nan)
    for f in range(F):
        v = pml[f]
        k = int(st["n_paths"][f])
        g_list[f, :k] = pm_values(v[:k].copy(), code.quant)
        assert (v[k:] == 0xFFFFFFFF).all()
    assert np.array_equal(st["L_used"], ref.L_used), "L_used"
    assert np.array_equal(st["crc_ok"], ref.crc_ok), "crc_ok"
    assert np.array_equal(st["n_paths"], ref.n_pm), "paths alive"
    bit_eq = (bits == ref.info).all(axis=1)
    if code.quant == O.F32:
        tol = PM_RTOL * np.maximum(1.0, np.abs(ref.pm))
        assert (np.abs(g_pm - ref.pm) <= tol).all(), "pm"
        lt = PM_RTOL * np.maximum(1.0, np.nan_to_num(np.abs(ref.pm_list)))
        d = np.abs(np.nan_to_num(g_list) - np.nan_to_num(ref.pm_list))
        bad = np.nonzero(~(d <= lt).all(axis=1))[0]
        assert len(bad) == 0, f"pm list: {len(bad)} frames, first {bad[:3]}: gpu {g_list[bad[:2]]} ref {ref.pm_list[bad[:2]]}"
        # decoded bits identical except on frames the oracle flags near-tie
        assert (bit_eq | (ref.near_tie == 1)).all(), "info bits"
    else:
        assert np.array_equal(g_pm, ref.pm), "pm"
        eq = (np.nan_to_num(g_list, nan=-1) == np.nan_to_num(ref.pm_list, nan=-1)).all(axis=1)
        bad = np.nonzero(~eq)[0]
        assert len(bad) == 0, f"pm list: {len(bad)} frames, first {bad[:3]}: gpu {g_list[bad[:2]]} ref {ref.pm_list[bad[:2]]}"
        assert bit_eq.all(), f"info bits: frames {np.nonzero(~bit_eq)[0][:5]}"
    exact = bool(bit_eq.all()) and np.array_equal(np.nan_to_num(g_list, nan=-1),
                                                   np.nan_to_num(ref.pm_list, nan=-1))
    return {"frames": F, "exact": exact, "fer_gpu": None, "escalated": int((ref.L_used > 1).sum())}
