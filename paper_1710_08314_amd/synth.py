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
