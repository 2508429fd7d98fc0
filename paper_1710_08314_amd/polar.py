"""Python binding of the gfx950 polar SCL decoder (libpolar_scl.so).

Argument marshalling only: every step of decoding, encoding and channel
generation runs in the library's HIP kernels.  PyTorch provides device memory
and the current stream.  The names follow the C ABI in include/polar_scl.h.
If the library is missing this module raises at import time; there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

# PyTorch first: its wheel carries its own HIP runtime, and the library must
# bind to the runtime PyTorch uses (loading the library first would put the
# system runtime under PyTorch, which then sees no GPU).
import torch  # noqa: F401

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpolar_scl.so")

F32, I16, I8 = 0, 1, 2
SC, CA_SCL, PA_SCL, FA_SCL = 0, 1, 2, 3
NODE_R0, NODE_R1, NODE_REP, NODE_SPC = 1, 2, 4, 8
NODE_ALL = 15
QUANT_NAMES = {"f32": F32, "i16": I16, "i8": I8}
ALGO_NAMES = {"sc": SC, "ca": CA_SCL, "pa": PA_SCL, "fa": FA_SCL}
ELEM_BYTES = {F32: 4, I16: 2, I8: 1}

ERRORS = {0: "success", -1: "invalid argument", -2: "unsupported configuration",
          -3: "out of memory", -4: "HIP runtime error",
          -5: "frozen set not usable for systematic encoding",
          -6: "no free serving slot or budget",
          -7: "batch exceeds the fixed device area of the allocation-free entry point"}
EAGAIN = -6


class PolarError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {ERRORS.get(code, 'unknown')} ({code})")
        self.code = code


class _Desc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_uint32), ("K", ctypes.c_uint32), ("frozen", ctypes.c_void_p),
                ("design_ebn0_db", ctypes.c_float), ("n_shorten", ctypes.c_uint32),
                ("crc_len", ctypes.c_uint32), ("crc_poly", ctypes.c_uint64),
                ("algo", ctypes.c_uint32), ("L", ctypes.c_uint32), ("L_max", ctypes.c_uint32),
                ("quant", ctypes.c_uint32), ("node_enable", ctypes.c_uint32),
                ("rep_max", ctypes.c_uint32), ("spc_max", ctypes.c_uint32),
                ("r1_max", ctypes.c_uint32), ("r0_max", ctypes.c_uint32),
                ("n_puncture", ctypes.c_uint32)]


class _Info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in (
        "N", "K", "crc_len", "n_tx", "k_data", "info_words", "code_words", "llr_bytes",
        "max_list", "n_ops", "n_r0", "n_r1", "n_rep", "n_spc", "n_leaf_frozen", "n_leaf_info",
        "lds_bytes")]


class _Opts(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("d_times", ctypes.c_void_p), ("reserved", ctypes.c_uint32 * 4)]


class _ServerCfg(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("max_inflight", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("budget_bytes", ctypes.c_uint64), ("slot_spill_bytes", ctypes.c_uint64)]


EXPORTS = ["polar_scl_plan", "polar_plan_destroy", "polar_plan_get_info", "polar_plan_get_frozen",
           "polar_plan_query",
           "polar_scl_decode_batch", "polar_scl_decode_batch_noalloc", "polar_encode", "polar_gen_data", "polar_channel",
           "polar_plan_stage_work", "polar_device_clock_khz", "polar_last_tier_ms",
           "polar_schedule_describe", "polar_graph_create", "polar_graph_launch",
           "polar_graph_destroy", "polar_server_create", "polar_server_submit",
           "polar_server_poll", "polar_server_inflight", "polar_server_destroy",
           "polar_serve_replay", "polar_plan_frame_bytes", "polar_quantize", "polar_strerror",
           "polar_version"]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1710_08314_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
    L.polar_scl_plan.argtypes = [ctypes.POINTER(_Desc), ctypes.POINTER(vp)]
    L.polar_plan_destroy.argtypes = [vp]
    L.polar_plan_get_info.argtypes = [vp, ctypes.POINTER(_Info)]
    L.polar_plan_get_frozen.argtypes = [vp, vp]
    L.polar_plan_query.argtypes = [ctypes.POINTER(_Desc), ctypes.POINTER(_Info), vp]
    L.polar_scl_decode_batch.argtypes = [vp, u32, vp, u32, vp, vp, vp, vp, vp, vp]
    L.polar_scl_decode_batch_noalloc.argtypes = [vp, u32, vp, u32, vp, vp, vp, vp, vp, vp]
    L.polar_encode.argtypes = [vp, vp, vp, u32, vp]
    L.polar_gen_data.argtypes = [vp, u64, u64, u32, vp, vp]
    L.polar_channel.argtypes = [vp, vp, u32, ctypes.c_float, i32, u64, u64, vp, vp]
    L.polar_plan_stage_work.argtypes = [vp, u32, ctypes.POINTER(ctypes.c_uint64)]
    L.polar_device_clock_khz.argtypes = [ctypes.POINTER(ctypes.c_uint32)]
    L.polar_last_tier_ms.argtypes = [ctypes.POINTER(ctypes.c_float)]
    L.polar_schedule_describe.argtypes = [vp, u32, ctypes.c_char_p, u32]
    L.polar_graph_create.argtypes = [vp, u32, vp, u32, vp, vp, vp, vp, vp, ctypes.POINTER(vp)]
    L.polar_graph_launch.argtypes = [vp, vp]
    L.polar_graph_destroy.argtypes = [vp]
    L.polar_server_create.argtypes = [ctypes.POINTER(_ServerCfg), ctypes.POINTER(vp)]
    L.polar_server_submit.argtypes = [vp, vp, u32, vp, u32, u32, vp, vp, vp, vp, u64,
                                      ctypes.POINTER(u32)]
    L.polar_plan_frame_bytes.argtypes = [vp, ctypes.POINTER(u64)]
    L.polar_quantize.argtypes = [vp, u32, i32, i32, vp, vp]
    L.polar_server_poll.argtypes = [vp, ctypes.POINTER(u64), u32, ctypes.POINTER(u32)]
    L.polar_server_inflight.argtypes = [vp, ctypes.POINTER(u32)]
    L.polar_server_destroy.argtypes = [vp]
    L.polar_serve_replay.argtypes = [vp, vp, u32, vp, u32, vp, vp, vp, vp, vp, vp, vp]
    L.polar_strerror.argtypes = [ctypes.c_int]
    L.polar_strerror.restype = ctypes.c_char_p
    L.polar_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("polar_strerror", "polar_version"):
            getattr(L, name).restype = ctypes.c_int
    return L


lib = _load()


def _check(rc: int, what: str):
    if rc != 0:
        raise PolarError(rc, what)


def _stream_ptr(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def pack_frozen(frozen: np.ndarray) -> np.ndarray:
    """uint8 mask (1 = frozen) -> ceil(N/32) little-endian words."""
    N = len(frozen)
    words = np.zeros((N + 31) // 32, dtype=np.uint32)
    for j in np.nonzero(frozen)[0]:
        words[j >> 5] |= np.uint32(1 << (j & 31))
    return words


def unpack_bits(words: np.ndarray, nbits: int) -> np.ndarray:
    """[..., W] uint32 words -> [..., nbits] uint8 bits (bit j = word j/32 bit j%32)."""
    w = np.ascontiguousarray(words, dtype=np.uint32)
    b = np.unpackbits(w.view(np.uint8), axis=-1, bitorder="little")
    return b[..., :nbits]


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """[..., n] 0/1 -> [..., ceil(n/32)] uint32."""
    bits = np.ascontiguousarray(bits, dtype=np.uint8)
    n = bits.shape[-1]
    W = (n + 31) // 32
    pad = np.zeros(bits.shape[:-1] + (W * 32,), dtype=np.uint8)
    pad[..., :n] = bits
    by = np.packbits(pad, axis=-1, bitorder="little")
    return by.view(np.uint32).reshape(bits.shape[:-1] + (W,))


@dataclass
class PlanInfo:
    N: int
    K: int
    crc_len: int
    n_tx: int
    k_data: int
    info_words: int
    code_words: int
    llr_bytes: int
    max_list: int
    n_ops: int
    n_r0: int
    n_r1: int
    n_rep: int
    n_spc: int
    n_leaf_frozen: int
    n_leaf_info: int
    lds_bytes: int


def _desc(N, K, crc_len, crc_poly, frozen, design_ebn0_db, n_shorten, algo, L, L_max, quant,
          node_enable, rep_max, spc_max, r1_max, r0_max, n_puncture=0):
    if isinstance(quant, str):
        quant = QUANT_NAMES[quant]
    if isinstance(algo, str):
        algo = ALGO_NAMES[algo]
    if rep_max is None:
        rep_max = 8 if quant == I8 else 0
    fw = pack_frozen(np.asarray(frozen, dtype=np.uint8)) if frozen is not None else None
    d = _Desc(N, K, fw.ctypes.data if fw is not None else None, float(design_ebn0_db), n_shorten,
              crc_len, crc_poly, algo, L, L_max, quant, node_enable, rep_max, spc_max, r1_max,
              r0_max, n_puncture)
    return d, fw, quant, algo


def plan_query(N, K, crc_len=0, crc_poly=0, frozen=None, design_ebn0_db=0.0, n_shorten=0,
               algo=CA_SCL, L=1, L_max=1, quant=F32, node_enable=NODE_ALL, rep_max=None,
               spc_max=4, r1_max=0, r0_max=0, n_puncture=0):
    """polar_plan_query: host-only planning -> (PlanInfo, frozen uint8 mask)."""
    d, fw, quant, algo = _desc(N, K, crc_len, crc_poly, frozen, design_ebn0_db, n_shorten, algo,
                               L, L_max, quant, node_enable, rep_max, spc_max, r1_max, r0_max,
                               n_puncture)
    inf = _Info()
    out = np.zeros((N + 31) // 32, dtype=np.uint32)
    _check(lib.polar_plan_query(ctypes.byref(d), ctypes.byref(inf), out.ctypes.data),
           "polar_plan_query")
    return PlanInfo(*[getattr(inf, f) for f, _ in _Info._fields_]), unpack_bits(out, N)


class Plan:
    """A code + decoder configuration (polar_scl_plan)."""

    def __init__(self, N, K, crc_len=0, crc_poly=0, frozen=None, design_ebn0_db=0.0,
                 n_shorten=0, algo=CA_SCL, L=1, L_max=1, quant=F32, node_enable=NODE_ALL,
                 rep_max=None, spc_max=4, r1_max=0, r0_max=0, n_puncture=0):
        d, self._fw, quant, algo = _desc(N, K, crc_len, crc_poly, frozen, design_ebn0_db,
                                         n_shorten, algo, L, L_max, quant, node_enable, rep_max,
                                         spc_max, r1_max, r0_max, n_puncture)
        h = ctypes.c_void_p()
        _check(lib.polar_scl_plan(ctypes.byref(d), ctypes.byref(h)), "polar_scl_plan")
        self._h = h
        self.quant, self.algo = quant, algo
        self.L, self.L_max = L, L_max
        inf = _Info()
        _check(lib.polar_plan_get_info(self._h, ctypes.byref(inf)), "polar_plan_get_info")
        self.info = PlanInfo(*[getattr(inf, f) for f, _ in _Info._fields_])

    @property
    def handle(self):
        return self._h

    def frame_bytes(self) -> int:
        """polar_plan_frame_bytes: bytes a frame in flight is charged by a server."""
        v = ctypes.c_uint64()
        _check(lib.polar_plan_frame_bytes(self._h, ctypes.byref(v)), "polar_plan_frame_bytes")
        return int(v.value)

    def stage_work(self, L: int) -> int:
        """Algorithmic element operations of one stage at list size L."""
        v = ctypes.c_uint64()
        _check(lib.polar_plan_stage_work(self._h, L, ctypes.byref(v)), "polar_plan_stage_work")
        return int(v.value)

    def frozen(self) -> np.ndarray:
        w = np.zeros(self.info.code_words, dtype=np.uint32)
        _check(lib.polar_plan_get_frozen(self._h, w.ctypes.data), "polar_plan_get_frozen")
        return unpack_bits(w, self.info.N)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.polar_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def llr_dtype(quant):
    import torch

    return {F32: torch.float32, I16: torch.int16, I8: torch.int8}[quant]


def device_clock_khz() -> int:
    v = ctypes.c_uint32()
    _check(lib.polar_device_clock_khz(ctypes.byref(v)), "polar_device_clock_khz")
    return int(v.value)


OPT_TIER_TIMING = 1
OPT_AUTOTUNE = 2
TIER_NAMES = ("sc", "list_a", "list_b", "plain", "classes")


def last_tier_ms():
    """polar_last_tier_ms: kernel durations of the last timed decode_batch."""
    v = (ctypes.c_float * 5)()
    _check(lib.polar_last_tier_ms(v), "polar_last_tier_ms")
    return dict(zip(TIER_NAMES, [float(x) for x in v]))


def schedule_describe(plans) -> str:
    """polar_schedule_describe: the class schedule used for this plan list."""
    arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
    buf = ctypes.create_string_buffer(4096)
    _check(lib.polar_schedule_describe(arr, len(plans), buf, len(buf)), "polar_schedule_describe")
    return buf.value.decode()


def _outputs(plans, llr, frames, n_frames, with_pm_lists):
    import torch

    dev = llr.device
    iw = max(p.info.info_words for p in plans)
    ml = max(p.info.max_list for p in plans)
    if frames is None:
        info = torch.empty((n_frames, iw), dtype=torch.int32, device=dev)
    else:
        tot = int(frames[:, 2].max().item()) + iw if n_frames else 0  # out_off column
        info = torch.zeros((max(tot, 1),), dtype=torch.int32, device=dev)
    status = torch.empty((n_frames, 8), dtype=torch.uint8, device=dev)
    pml = torch.empty((n_frames, ml), dtype=torch.int32, device=dev) if with_pm_lists else None
    return info, status, pml


class Graph:
    """polar_graph_*: one decode of fixed buffers captured into a HIP graph.
    The output tensors are allocated here and rewritten by every replay."""

    def __init__(self, plans, llr, frames=None, n_frames=None, with_pm_lists=False, schedule=0):
        if isinstance(plans, Plan):
            plans = [plans]
        if n_frames is None:
            n_frames = frames.shape[0] if frames is not None else llr.shape[0]
        self._keep = (plans, llr, frames)
        self.info, self.status, self.pm_lists = _outputs(plans, llr, frames, n_frames,
                                                         with_pm_lists)
        arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
        opts = _Opts(schedule, 0, None)
        h = ctypes.c_void_p()
        _check(lib.polar_graph_create(arr, len(plans), _dptr(frames), n_frames, _dptr(llr),
                                      _dptr(self.info), _dptr(self.status), _dptr(self.pm_lists),
                                      ctypes.byref(opts), ctypes.byref(h)), "polar_graph_create")
        self._h = h

    def launch(self, stream=None):
        _check(lib.polar_graph_launch(self._h, _stream_ptr(stream)), "polar_graph_launch")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.polar_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """polar_server_*: continuous batching over `n_slots` HIP streams."""

    def __init__(self, n_slots=4, max_batch=4096, max_inflight=16384, budget_bytes=0,
                 slot_spill_bytes=0):
        cfg = _ServerCfg(n_slots, max_batch, max_inflight, 0, budget_bytes, slot_spill_bytes)
        h = ctypes.c_void_p()
        _check(lib.polar_server_create(ctypes.byref(cfg), ctypes.byref(h)), "polar_server_create")
        self._h = h

    def submit(self, plans, frames, first, count, llr, info, status, tag=0, plan_idx=None):
        """Admit frames [first, first + count); False when no slot or budget.
        plan_idx: optional host array of the batch's plan indices (byte budget)."""
        arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
        slot = ctypes.c_uint32()
        pi = np.ascontiguousarray(plan_idx, dtype=np.uint32) if plan_idx is not None else None
        rc = lib.polar_server_submit(self._h, arr, len(plans), _dptr(frames), first, count,
                                     pi.ctypes.data if pi is not None else None,
                                     _dptr(llr), _dptr(info), _dptr(status), tag,
                                     ctypes.byref(slot))
        if rc == EAGAIN:
            return False
        _check(rc, "polar_server_submit")
        return True

    def poll(self, max_tags=64):
        tags = (ctypes.c_uint64 * max_tags)()
        n = ctypes.c_uint32()
        _check(lib.polar_server_poll(self._h, tags, max_tags, ctypes.byref(n)), "polar_server_poll")
        return [int(tags[i]) for i in range(n.value)]

    def inflight(self):
        v = ctypes.c_uint32()
        _check(lib.polar_server_inflight(self._h, ctypes.byref(v)), "polar_server_inflight")
        return int(v.value)

    def replay(self, plans, frames, arrival_us, llr, info, status, plan_of=None):
        """polar_serve_replay: returns (completion times in us, stats dict).
        plan_of: optional host array of every request's plan index (byte budget)."""
        arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
        arrival = np.ascontiguousarray(arrival_us, dtype=np.float64)
        n = len(arrival)
        done = np.zeros(n, dtype=np.float64)
        stats = np.zeros(5, dtype=np.float64)
        po = np.ascontiguousarray(plan_of, dtype=np.uint32) if plan_of is not None else None
        _check(lib.polar_serve_replay(self._h, arr, len(plans), _dptr(frames), n,
                                      arrival.ctypes.data, po.ctypes.data if po is not None else None,
                                      _dptr(llr), _dptr(info), _dptr(status),
                                      done.ctypes.data, stats.ctypes.data), "polar_serve_replay")
        return done, {"batches": int(stats[0]), "mean_batch": float(stats[1]),
                      "peak_inflight": int(stats[2]), "session_us": float(stats[3]),
                      "peak_inflight_bytes": int(stats[4])}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.polar_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decode_batch(plans, llr, frames=None, n_frames=None, with_pm_lists=False, schedule=0,
                 stream=None, times=None, tier_timing=False, autotune=False):
    """polar_scl_decode_batch.  `plans`: Plan or list of Plan; `llr`: device
    tensor (uniform batch: [F, n_tx] of the plan's dtype; with `frames`: any
    byte buffer).  Returns (info [F, info_words] int32, status [F, 8] uint8,
    pm_lists [F, max_list] int32 or None)."""
    if isinstance(plans, Plan):
        plans = [plans]
    if n_frames is None:
        n_frames = frames.shape[0] if frames is not None else llr.shape[0]
    info, status, pml = _outputs(plans, llr, frames, n_frames, with_pm_lists)
    arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
    flags = (OPT_TIER_TIMING if tier_timing else 0) | (OPT_AUTOTUNE if autotune else 0)
    opts = _Opts(schedule, flags, times.data_ptr() if times is not None else None)
    _check(lib.polar_scl_decode_batch(arr, len(plans), _dptr(frames), n_frames, _dptr(llr),
                                      _dptr(info), _dptr(status), _dptr(pml),
                                      ctypes.byref(opts), _stream_ptr(stream)),
           "polar_scl_decode_batch")
    return info, status, pml


def decode_batch_noalloc(plans, llr, info, status, pm_lists=None, frames=None, n_frames=None,
                         schedule=0, stream=None):
    """polar_scl_decode_batch_noalloc: the decode of decode_batch into output
    tensors the caller provides (info, status and optional pm_lists, shaped as
    decode_batch returns them), using the library's fixed device area."""
    if isinstance(plans, Plan):
        plans = [plans]
    if n_frames is None:
        n_frames = frames.shape[0] if frames is not None else llr.shape[0]
    arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
    opts = _Opts(schedule, 0, None)
    _check(lib.polar_scl_decode_batch_noalloc(arr, len(plans), _dptr(frames), n_frames,
                                              _dptr(llr), _dptr(info), _dptr(status),
                                              _dptr(pm_lists), ctypes.byref(opts),
                                              _stream_ptr(stream)),
           "polar_scl_decode_batch_noalloc")


def encode(plan: Plan, data, stream=None):
    """polar_encode: data [F, info_words] int32 (device) -> code [F, code_words]."""
    import torch

    F = data.shape[0]
    code = torch.empty((F, plan.info.code_words), dtype=torch.int32, device=data.device)
    _check(lib.polar_encode(plan.handle, _dptr(data), _dptr(code), F, _stream_ptr(stream)),
           "polar_encode")
    return code


def gen_data(plan: Plan, seed: int, frame0: int, n_frames: int, device="cuda", stream=None):
    import torch

    out = torch.empty((n_frames, plan.info.info_words), dtype=torch.int32, device=device)
    _check(lib.polar_gen_data(plan.handle, seed, frame0, n_frames, _dptr(out),
                              _stream_ptr(stream)), "polar_gen_data")
    return out


def channel(plan: Plan, code, ebn0_db: float, seed: int, frame0: int, frac_bits=None,
            stream=None):
    import torch

    if frac_bits is None:
        frac_bits = {I8: 2, I16: 3}.get(plan.quant, 0)
    F = code.shape[0]
    llr = torch.empty((F, plan.info.n_tx), dtype=llr_dtype(plan.quant), device=code.device)
    _check(lib.polar_channel(plan.handle, _dptr(code), F, float(ebn0_db), int(frac_bits), seed,
                             frame0, _dptr(llr), _stream_ptr(stream)), "polar_channel")
    return llr


def quantize(llr, quant, frac_bits=None, stream=None):
    """polar_quantize: float32 device LLRs -> the quant's type (new tensor)."""
    import torch

    if isinstance(quant, str):
        quant = QUANT_NAMES[quant]
    if frac_bits is None:
        frac_bits = {I8: 2, I16: 3}.get(quant, 0)
    src = llr.contiguous()
    out = torch.empty(src.shape, dtype=llr_dtype(quant), device=src.device)
    _check(lib.polar_quantize(_dptr(src), src.numel(), quant, int(frac_bits), _dptr(out),
                              _stream_ptr(stream)), "polar_quantize")
    return out


def status_fields(status):
    """Split a [F, 8] uint8 status tensor (host numpy) into named arrays."""
    st = np.ascontiguousarray(status)
    return {"crc_ok": st[:, 0].astype(np.int32), "L_used": st[:, 1].astype(np.int32),
            "n_paths": st[:, 2].astype(np.int32), "near_tie": (st[:, 3] & 1).astype(np.int32),
            "pm_bits": st[:, 4:8].copy().view(np.uint32).reshape(-1)}
