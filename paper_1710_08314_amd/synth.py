"""Seeded synthetic inputs for the decoder workloads (host side).

This module only draws random numbers and states the workload shapes; it holds
none of the decoding method's arithmetic (no encoding, CRC, quantisation or
decoding).  Both the CPU oracle's tests and the benchmark's CPU leg build
their frames from what it returns.

Per frame the Monte-Carlo chain of the paper (Sec. II-C: BPSK over AWGN) needs
* K - c i.i.d. Bernoulli(1/2) data bits, and
* N - S i.i.d. standard normal noise samples.
Streams are addressable by (seed, block) through ``numpy.random.SeedSequence``
so that any block of frames can be regenerated on its own.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BLOCK = 1024  # frames per independently seeded block


def _block_rng(seed: int, block: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(np.random.SeedSequence([int(seed), int(block)])))


def frames(seed: int, first: int, count: int, k_data: int, n_tx: int):
    """Data bits [count, k_data] (uint8) and noise [count, n_tx] (float64)."""
    bits = np.zeros((count, k_data), dtype=np.uint8)
    noise = np.zeros((count, n_tx), dtype=np.float64)
    f = first
    while f < first + count:
        blk = f // BLOCK
        rng = _block_rng(seed, blk)
        b = rng.integers(0, 2, size=(BLOCK, k_data), dtype=np.uint8)
        z = rng.standard_normal(size=(BLOCK, n_tx))
        lo = f - blk * BLOCK
        hi = min(BLOCK, first + count - blk * BLOCK)
        bits[f - first:f - first + hi - lo] = b[lo:hi]
        noise[f - first:f - first + hi - lo] = z[lo:hi]
        f += hi - lo
    return bits, noise


def sigma_for(ebn0_db: float, k_data: int, n_tx: int) -> float:
    """AWGN standard deviation for BPSK at Eb/N0 with rate R = k_data / n_tx:
    sigma^2 = 1 / (2 R Eb/N0)."""
    r = k_data / n_tx
    return math.sqrt(1.0 / (2.0 * r * 10.0 ** (ebn0_db / 10.0)))


@dataclass
class Workload:
    """One synthetic decoding workload (a code, a decoder and channel points)."""

    name: str
    N: int
    K: int            # |A| including the CRC bits
    crc_len: int
    crc_poly: int
    design_db: float  # Bhattacharyya design Eb/N0
    quant: str        # "f32" | "i16" | "i8"
    algo: str         # "sc" | "ca" | "pa" | "fa"
    L: int
    L_max: int
    ebn0_db: list = field(default_factory=list)
    frames: int = 0
    seed: int = 0
    rep_max: int = 0
    spc_max: int = 4

    @property
    def k_data(self) -> int:
        return self.K - self.crc_len


# The workloads of the paper's experiments that the decoder reproduces.
# 1. CA-SCL on a (256, 120 + CRC-8) code, the small case.
C1 = Workload("ca_scl_n256_k128_crc8_l4_f32", 256, 128, 8, 0x07, 2.0, "f32", "ca", 4, 4,
              [2.5], 1000, 0)
# 2. The paper's headline code (2048, 1723 incl. CRC-32), fully adaptive
#    L = 1 -> 32, 8-bit fixed point with REP8- and SPC4 (Sec. III-B3, Table III).
C2 = Workload("fa_sscl_n2048_k1723_crc32_lmax32_i8", 2048, 1723, 32, 0x04C11DB7, 4.5, "i8",
              "fa", 1, 32, [3.5, 4.0, 4.5], 1_000_000, 2000, rep_max=8)
# 5. Quantisation sweep (1024, 488 + CRC-24), L = 8.
C5 = Workload("ca_scl_n1024_k512_crc24_l8", 1024, 512, 24, 0x1864CFB, 2.5, "f32", "ca", 8, 8,
              [1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0], 10_000_000, 5000)


# 3. Batched uneven launch: every frame draws its own code and decoder.
C3_N = (128, 256, 512, 1024, 2048)
C3_RATES = (1 / 4, 1 / 3, 1 / 2, 2 / 3, 5 / 6)
C3_L = (2, 8, 32)
C3_CRC = (11, 0x621)
C3_DESIGN_DB = 2.5
C3_SHORTENED = 0.2  # fraction of frames shortened by S ~ U{1 .. N/4}


def uneven_batch(seed: int, n: int):
    """Per-frame draws of the uneven batch: N, rate, L, shortening S and
    Eb/N0 ~ U[1, 4] dB.  Returns (codes, code_idx, ebn0): `codes` lists the
    distinct (N, K, L, S) with K = round(rate (N - S)) = |A| including the
    CRC, `code_idx[f]` the code of frame f."""
    rng = np.random.Generator(np.random.Philox(np.random.SeedSequence([int(seed), 0xC3])))
    N = rng.choice(np.array(C3_N), size=n)
    r = rng.integers(0, len(C3_RATES), size=n)
    L = rng.choice(np.array(C3_L), size=n)
    short = rng.random(n) < C3_SHORTENED
    S = np.where(short, rng.integers(1, N // 4 + 1), 0)
    ebn0 = rng.uniform(1.0, 4.0, size=n)
    K = np.rint(np.array(C3_RATES)[r] * (N - S)).astype(np.int64)
    key = np.stack([N, K, L, S], axis=1)
    codes, code_idx = np.unique(key, axis=0, return_inverse=True)
    return [tuple(int(v) for v in c) for c in codes], code_idx.reshape(-1), ebn0


def frame_draws(seed: int, f: int, k_data: int, n_tx: int):
    """Data bits [k_data] and noise [n_tx] of frame f alone (a generator per
    (seed, frame), for batches whose frames all differ in size)."""
    rng = np.random.Generator(np.random.Philox(np.random.SeedSequence([int(seed), 0xF, int(f)])))
    return rng.integers(0, 2, size=k_data, dtype=np.uint8), rng.standard_normal(size=n_tx)


# 4. Served decoding: Poisson arrivals of requests of mixed sizes.
C4_N = (32, 64, 128, 256, 512, 1024)
C4_CRC = (11, 0x621)
C4_L_MAX = 8
C4_DESIGN_DB = 1.5
C4_RATES_MREQ = (0.5, 1.0, 2.0, 4.0, 8.0)


def served_requests(seed: int, n: int, rate_per_s: float):
    """n requests: N with P(N) proportional to 1/N, K ~ U{12 .. N/2} (|A|
    including CRC-11), Eb/N0 ~ U[0, 3] dB and Poisson arrival times (us).
    Returns (codes, code_idx, ebn0, arrival_us) with `codes` the distinct
    (N, K)."""
    rng = np.random.Generator(np.random.Philox(np.random.SeedSequence([int(seed), 0xC4])))
    w = 1.0 / np.array(C4_N, dtype=np.float64)
    N = rng.choice(np.array(C4_N), size=n, p=w / w.sum())
    K = rng.integers(12, N // 2 + 1)
    ebn0 = rng.uniform(0.0, 3.0, size=n)
    gaps = rng.exponential(1e6 / rate_per_s, size=n)
    arrival = np.cumsum(gaps) - gaps[0]
    key = np.stack([N, K], axis=1)
    codes, code_idx = np.unique(key, axis=0, return_inverse=True)
    return [tuple(int(v) for v in c) for c in codes], code_idx.reshape(-1), ebn0, arrival
