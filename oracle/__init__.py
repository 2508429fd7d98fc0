"""CPU oracle for flexible CRC-aided SCL polar decoding -- TEST INFRASTRUCTURE.

Thin ctypes binding over ``oracle/oracle.cpp`` (a plain, literal C++
implementation of Algorithm 1 of Leonardon et al., arXiv:1710.08314, with the
dedicated nodes of Sec. II-B3, the CRC selection of Sec. II-B4 / IV-B and the
adaptive schedules of Sec. II-B5).  Only ``tests/``, ``__graft_entry__.smoke``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package; the
product decoder never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
# A build of a modified copy of oracle.cpp may be loaded instead, for the
# mutation check of the pins (tests/oracle_mutations.py); never set otherwise.
_LIB_OVERRIDE = os.environ.get("POLAR_ORACLE_LIB_OVERRIDE")

F32, I16, I8, F64 = 0, 1, 2, 3
SC, CA_SCL, PA_SCL, FA_SCL = 0, 1, 2, 3
NODE_R0, NODE_R1, NODE_REP, NODE_SPC = 1, 2, 4, 8
NODE_ALL = NODE_R0 | NODE_R1 | NODE_REP | NODE_SPC
KIND_NAMES = {0: "LEAF_F", 1: "LEAF_I", 2: "R0", 3: "R1", 4: "REP", 5: "SPC"}
DTYPES = {F32: np.float32, I16: np.int16, I8: np.int8, F64: np.float64}
QMAX = {I16: 32767, I8: 127}


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (-O2, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-pthread", "-o", tmp, _SRC]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int32), ("K", ctypes.c_int32), ("crc_len", ctypes.c_int32),
        ("crc_poly", ctypes.c_uint64), ("frozen", ctypes.c_void_p), ("S", ctypes.c_int32),
        ("quant", ctypes.c_int32), ("algo", ctypes.c_int32), ("L", ctypes.c_int32),
        ("L_max", ctypes.c_int32), ("node_enable", ctypes.c_int32), ("rep_max", ctypes.c_int32),
        ("spc_max", ctypes.c_int32), ("r1_max", ctypes.c_int32), ("r0_max", ctypes.c_int32),
        ("P", ctypes.c_int32),
    ]


class _Status(ctypes.Structure):
    _fields_ = [("crc_ok", ctypes.c_int32), ("L_used", ctypes.c_int32),
                ("near_tie", ctypes.c_int32), ("n_pm", ctypes.c_int32), ("pm", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = ctypes.CDLL(_LIB)
        vp, i32, u64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_double
        L.orc_logz_z0.argtypes = [i32, dbl, vp]
        L.orc_construct.argtypes = [i32, i32, i32, i32, dbl, vp]
        L.orc_construct.restype = i32
        L.orc_construct_lz0.argtypes = [i32, i32, i32, dbl, vp]
        L.orc_construct_lz0.restype = i32
        L.orc_construct_p.argtypes = [i32, i32, i32, i32, i32, dbl, vp]
        L.orc_construct_p.restype = i32
        L.orc_construct_lz0p.argtypes = [i32, i32, i32, i32, dbl, vp]
        L.orc_construct_lz0p.restype = i32
        L.orc_fg.argtypes = [i32, i32, dbl, dbl, i32]
        L.orc_fg.restype = dbl
        L.orc_transform.argtypes = [i32, vp, vp]
        L.orc_encode.argtypes = [i32, vp, vp, vp]
        L.orc_crc.argtypes = [vp, i32, i32, u64]
        L.orc_crc.restype = u64
        L.orc_attach_crc.argtypes = [vp, i32, i32, u64, vp]
        L.orc_bpsk_awgn_llr.argtypes = [vp, i32, vp, dbl, vp]
        L.orc_quantize.argtypes = [vp, i32, i32, i32, vp]
        L.orc_decode.argtypes = [ctypes.POINTER(_Cfg), vp, vp, vp, vp, ctypes.POINTER(_Status)]
        L.orc_decode.restype = i32
        L.orc_decode_batch.argtypes = [ctypes.POINTER(_Cfg), i32, vp, ctypes.c_int64, vp, vp, vp,
                                       vp, i32]
        L.orc_decode_batch.restype = i32
        L.orc_nodes.argtypes = [ctypes.POINTER(_Cfg), vp, vp, vp, i32]
        L.orc_make_frames.argtypes = [ctypes.POINTER(_Cfg), i32, vp, vp, dbl, i32, vp]
        L.orc_make_frames.restype = i32
        L.orc_nodes.restype = i32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------- construction
def logz_from_z0(n: int, lz0: float) -> np.ndarray:
    out = np.zeros(1 << n, dtype=np.float64)
    lib().orc_logz_z0(n, float(lz0), _p(out))
    return out


def construct(N: int, K: int, S: int, crc_len: int, design_ebn0_db: float,
              P: int = 0) -> np.ndarray:
    """Frozen mask (uint8, 1 = frozen) by the Bhattacharyya reading; K = |A|;
    S shortened (last) and P punctured (first) codeword positions."""
    fz = np.zeros(N, dtype=np.uint8)
    rc = lib().orc_construct_p(N, K, S, P, crc_len, float(design_ebn0_db), _p(fz))
    if rc:
        raise ValueError("bad construction arguments")
    return fz


def construct_lz0(N: int, K: int, S: int, lz0: float, P: int = 0) -> np.ndarray:
    """Frozen mask from an explicit log Z0 of the underlying channel."""
    fz = np.zeros(N, dtype=np.uint8)
    if lib().orc_construct_lz0p(N, K, S, P, float(lz0), _p(fz)):
        raise ValueError("bad construction arguments")
    return fz


def fg(quant: int, op: str, a: float, b: float, s: int = 0) -> float:
    """The oracle's f (op="f") or g (op="g") on one pair of values."""
    return float(lib().orc_fg(quant, 1 if op == "g" else 0, float(a), float(b), int(s)))


def transform(v: np.ndarray) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.uint8)
    x = np.zeros_like(v)
    lib().orc_transform(len(v), _p(v), _p(x))
    return x


def encode(frozen: np.ndarray, b: np.ndarray) -> np.ndarray:
    frozen = np.ascontiguousarray(frozen, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    x = np.zeros(len(frozen), dtype=np.uint8)
    lib().orc_encode(len(frozen), _p(frozen), _p(b), _p(x))
    return x


def crc(bits: np.ndarray, c: int, poly: int) -> int:
    bits = np.ascontiguousarray(bits, dtype=np.uint8)
    return int(lib().orc_crc(_p(bits), len(bits), c, poly))


def attach_crc(data: np.ndarray, c: int, poly: int) -> np.ndarray:
    data = np.ascontiguousarray(data, dtype=np.uint8)
    b = np.zeros(len(data) + c, dtype=np.uint8)
    lib().orc_attach_crc(_p(data), len(data), c, poly, _p(b))
    return b


def bpsk_awgn_llr(x: np.ndarray, noise: np.ndarray, sigma: float) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.uint8)
    noise = np.ascontiguousarray(noise, dtype=np.float64)
    out = np.zeros(len(x), dtype=np.float64)
    lib().orc_bpsk_awgn_llr(_p(x), len(x), _p(noise), float(sigma), _p(out))
    return out


def quantize(llr: np.ndarray, quant: int, frac: int) -> np.ndarray:
    llr = np.ascontiguousarray(llr, dtype=np.float64)
    out = np.zeros(len(llr), dtype=DTYPES[quant])
    lib().orc_quantize(_p(llr), len(llr), quant, frac, _p(out))
    return out


# -------------------------------------------------------------------- decoding
@dataclass
class Code:
    """A decoder configuration for the oracle (mirrors the plan parameters)."""

    N: int
    K: int  # |A| including the CRC bits
    frozen: np.ndarray
    crc_len: int = 0
    crc_poly: int = 0
    S: int = 0
    quant: int = F32
    algo: int = CA_SCL
    L: int = 1
    L_max: int = 1
    node_enable: int = NODE_ALL
    rep_max: int = 0
    spc_max: int = 4
    r1_max: int = 0
    r0_max: int = 0
    P: int = 0  # punctured: the first P codeword positions are not sent

    def cfg(self) -> _Cfg:
        self._fz = np.ascontiguousarray(self.frozen, dtype=np.uint8)
        return _Cfg(self.N, self.K, self.crc_len, self.crc_poly, self._fz.ctypes.data, self.S,
                    self.quant, self.algo, self.L, self.L_max, self.node_enable, self.rep_max,
                    self.spc_max, self.r1_max, self.r0_max, self.P)

    @property
    def n_tx(self) -> int:
        return self.N - self.S - self.P

    @property
    def k_data(self) -> int:
        return self.K - self.crc_len

    def max_list(self) -> int:
        if self.algo == SC:
            return 1
        if self.algo == CA_SCL:
            return self.L
        return self.L_max


@dataclass
class Result:
    info: np.ndarray      # [F, K - c] uint8
    xhat: np.ndarray      # [F, N] uint8
    pm_list: np.ndarray   # [F, Lmax] float64 (nan past n_pm)
    crc_ok: np.ndarray
    L_used: np.ndarray
    near_tie: np.ndarray
    n_pm: np.ndarray
    pm: np.ndarray


def decode(code: Code, llr: np.ndarray, threads: int = 1) -> Result:
    """Decode a [F, N - S] array of LLRs of the mode's dtype."""
    llr = np.ascontiguousarray(llr, dtype=DTYPES[code.quant])
    if llr.ndim == 1:
        llr = llr[None, :]
    F = llr.shape[0]
    assert llr.shape[1] == code.n_tx
    lm = code.max_list()
    info = np.zeros((F, code.k_data), dtype=np.uint8)
    xhat = np.zeros((F, code.N), dtype=np.uint8)
    pml = np.full((F, lm), np.nan, dtype=np.float64)
    st = (_Status * max(F, 1))()
    cfg = code.cfg()
    rc = lib().orc_decode_batch(ctypes.byref(cfg), F, _p(llr), llr.strides[0], _p(info), _p(xhat),
                                _p(pml), ctypes.cast(st, ctypes.c_void_p), int(threads))
    if rc:
        raise ValueError(f"oracle rejected the configuration ({rc})")
    arr = np.frombuffer(st, dtype=np.dtype([("crc_ok", "<i4"), ("L_used", "<i4"),
                                             ("near_tie", "<i4"), ("n_pm", "<i4"),
                                             ("pm", "<f8")]), count=F)
    for f in range(F):
        pml[f, arr["n_pm"][f]:] = np.nan
    return Result(info, xhat, pml, arr["crc_ok"].copy(), arr["L_used"].copy(),
                  arr["near_tie"].copy(), arr["n_pm"].copy(), arr["pm"].copy())


def nodes(code: Code):
    """Pre-order dedicated-node decomposition: list of (kind name, start, size)."""
    cap = 2 * code.N
    k = np.zeros(cap, np.int32)
    s = np.zeros(cap, np.int32)
    z = np.zeros(cap, np.int32)
    cfg = code.cfg()
    cnt = lib().orc_nodes(ctypes.byref(cfg), _p(k), _p(s), _p(z), cap)
    return [(KIND_NAMES[int(k[i])], int(s[i]), int(z[i])) for i in range(cnt)]


def default_frac(quant: int) -> int:
    return {I8: 2, I16: 3}.get(quant, 0)


def make_frames(code: Code, data: np.ndarray, noise: np.ndarray, sigma: float,
                frac: int | None = None) -> np.ndarray:
    """CRC + systematic encoding + BPSK/AWGN + quantisation of data [F, K - c]
    with noise [F, N - S]: LLRs [F, N - S] of the mode's dtype (batched in C)."""
    frac = default_frac(code.quant) if frac is None else frac
    data = np.ascontiguousarray(data, dtype=np.uint8)
    noise = np.ascontiguousarray(noise, dtype=np.float64)
    F = data.shape[0]
    out = np.zeros((F, code.n_tx), dtype=DTYPES[code.quant])
    cfg = code.cfg()
    lib().orc_make_frames(ctypes.byref(cfg), F, _p(data), _p(noise), float(sigma), frac, _p(out))
    return out


def make_llr(code: Code, x_tx: np.ndarray, noise: np.ndarray, sigma: float,
             frac: int | None = None) -> np.ndarray:
    """BPSK/AWGN LLRs for transmitted bits [F, N - S], quantised to the mode."""
    frac = default_frac(code.quant) if frac is None else frac
    F = x_tx.shape[0]
    out = np.zeros((F, code.n_tx), dtype=DTYPES[code.quant])
    for f in range(F):
        l = bpsk_awgn_llr(x_tx[f], noise[f], sigma)
        out[f] = quantize(l, code.quant, frac)
    return out
