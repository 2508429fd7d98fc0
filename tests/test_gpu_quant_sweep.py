"""Quantisation sweep of the (1024, 488 + CRC-24) code, CA-SCL L = 8, Bhattacharyya
design at 2.5 dB: float32, saturated int16 and saturated int8 LLRs at Eb/N0 =
1.0, 1.5, ..., 4.0 dB (the fixed-point study of Sec. III-B3).

Per point the GPU decodes a host-made batch; the oracle decodes every 20th
frame of it.  Those frames must decode identically on both sides (exactly in
the integer modes; bits equal except oracle-flagged near-ties in float32), and
the frame error rate of the whole GPU batch must agree with the oracle's on
its subset within Monte-Carlo 95% (Wilson) intervals."""
import concurrent.futures as cf
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_1710_08314_amd import synth
from tests.gpu_util import gpu_plan, oracle_code, pm_values, PM_RTOL

pytestmark = pytest.mark.gpu

FRAMES = 40_000
SUB = 20
CHUNK = 8192
POINTS = [1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0]
QUANTS = {"f32": O.F32, "i16": O.I16, "i8": O.I8}


def wilson(k, n, z=1.96):
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return max(0.0, c - h), min(1.0, c + h)


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _inputs(code, seed, ebn0):
    sigma = synth.sigma_for(ebn0, code.k_data, code.n_tx)
    data = np.zeros((FRAMES, code.k_data), dtype=np.uint8)
    llr = np.zeros((FRAMES, code.n_tx), dtype=O.DTYPES[code.quant])

    def chunk(i):
        lo, hi = i * CHUNK, min(FRAMES, (i + 1) * CHUNK)
        b, z = synth.frames(seed, lo, hi - lo, code.k_data, code.n_tx)
        data[lo:hi] = b
        llr[lo:hi] = O.make_frames(code, b, z, sigma)

    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(chunk, range((FRAMES + CHUNK - 1) // CHUNK)))
    return data, llr


@pytest.mark.parametrize("quant", list(QUANTS))
def test_quant_sweep_fer(quant):
    import torch
    from paper_1710_08314_amd import polar as P

    q = QUANTS[quant]
    fz = O.construct(1024, 512, 0, 24, 2.5)
    code = oracle_code(1024, 512, 24, 0x1864CFB, fz, quant=q, algo="ca", L=8)
    plan = gpu_plan(code)
    threads = min(16, os.cpu_count() or 1)
    for pt, ebn0 in enumerate(POINTS):
        data, llr = _inputs(code, 5000 + pt, ebn0)
        info, status, _ = P.decode_batch(plan, torch.from_numpy(llr).cuda())
        torch.cuda.synchronize()
        bits = P.unpack_bits(info.cpu().numpy().view(np.uint32), code.k_data)
        st = P.status_fields(status.cpu().numpy())
        sub = np.arange(0, FRAMES, SUB)
        ref = O.decode(code, llr[sub], threads=threads)
        # the subset frame by frame
        eq = (bits[sub] == ref.info).all(axis=1)
        g_pm = pm_values(st["pm_bits"][sub], code.quant)
        assert np.array_equal(st["near_tie"][sub], ref.near_tie), f"{quant} {ebn0} dB: near-tie"
        if q == O.F32:
            # bits may differ only on near-tie frames; metrics always within tolerance
            assert (eq | (ref.near_tie == 1)).all(), f"{quant} {ebn0} dB: info bits"
            tol = PM_RTOL * np.maximum(1.0, np.abs(ref.pm))
            assert (np.abs(g_pm - ref.pm) <= tol).all(), f"{quant} {ebn0} dB: path metric"
            assert np.array_equal(st["crc_ok"][sub], ref.crc_ok)
        else:
            assert eq.all(), f"{quant} {ebn0} dB: info bits"
            assert np.array_equal(g_pm, ref.pm), f"{quant} {ebn0} dB: path metric"
            assert np.array_equal(st["crc_ok"][sub], ref.crc_ok)
        # error rates: whole GPU batch vs the oracle's subset
        fe_gpu = (bits != data).any(axis=1)
        fe_orc = (ref.info != data[sub]).any(axis=1)
        g_lo, g_hi = wilson(int(fe_gpu.sum()), FRAMES)
        o_lo, o_hi = wilson(int(fe_orc.sum()), len(sub))
        ber = float((bits != data).mean())
        print(f"{quant} {ebn0:.1f} dB FER gpu {fe_gpu.mean():.3e} [{g_lo:.2e}, {g_hi:.2e}] "
              f"oracle {fe_orc.mean():.3e} [{o_lo:.2e}, {o_hi:.2e}] BER gpu {ber:.3e}",
              flush=True)
        assert g_lo <= o_hi and o_lo <= g_hi, f"{quant} {ebn0} dB: FER intervals disjoint"
