"""The allocation-free decode entry point (polar_scl_decode_batch_noalloc)
against polar_scl_decode_batch on the same inputs: two calls in a row, the
second with a smaller batch, each compared element by element (decoded bits,
status words, path-metric lists).  The two entry points run the same kernels;
the allocation-free one cuts its persistent grids to its fixed device area,
which must not change any frame's result.

Cases: the (2048, 1691 + CRC-32) FA-SSCL L = 1 -> 32 int8 batch (per-lane
stages with spill regions, grids cut), a multi-plan fixed-list int16 batch
(class schedule, plan table written into the fixed area), and a float32
CA-SCL batch through the plain one-launch schedule."""
import numpy as np
import pytest

from tests.gpu_util import gpu_plan, uneven_inputs

pytestmark = pytest.mark.gpu


def _need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _both(plans, llr, frames=None, n_frames=None, schedule=0):
    """Outputs of the allocating and the allocation-free entry point."""
    import torch
    from paper_1710_08314_amd import polar as P

    if isinstance(plans, P.Plan):
        plans = [plans]
    info, status, pml = P.decode_batch(plans, llr, frames=frames, n_frames=n_frames,
                                       with_pm_lists=True, schedule=schedule)
    # a multi-plan batch writes each frame's own words of a shared buffer, which
    # decode_batch zero-fills; elsewhere every output word is written
    info2 = torch.zeros_like(info) if frames is not None else torch.full_like(info, -1)
    status2 = torch.full_like(status, 0xAA)
    pml2 = torch.full_like(pml, -1)
    P.decode_batch_noalloc(plans, llr, info2, status2, pml2, frames=frames, n_frames=n_frames,
                           schedule=schedule)
    torch.cuda.synchronize()
    return [(a.cpu().numpy(), b.cpu().numpy()) for a, b in
            ((info, info2), (status, status2), (pml, pml2))]


def _assert_same(pairs, what):
    for name, (a, b) in zip(("info bits", "status", "pm lists"), pairs):
        bad = np.nonzero((a != b).reshape(a.shape[0], -1).any(axis=1))[0]
        assert len(bad) == 0, f"{what}: {name} differ on {len(bad)} frames, first {bad[:5]}"


def test_noalloc_headline_two_calls():
    _need_gpu()
    from paper_1710_08314_amd import polar as P

    plan = P.Plan(2048, 1723, 32, 0x04C11DB7, design_ebn0_db=4.5, algo=P.FA_SCL, L=1, L_max=32,
                  quant=P.I8)
    for n, seed in ((1 << 17, 11), (3000, 12)):
        print(f"headline FA int8, {n} frames", flush=True)
        data = P.gen_data(plan, seed, 0, n)
        llr = P.channel(plan, P.encode(plan, data), 3.5, seed + 100, 0)
        pairs = _both(plan, llr)
        _assert_same(pairs, f"headline, {n} frames")
        st = P.status_fields(pairs[1][1])
        assert (st["L_used"] > 1).any(), "the batch reaches the list stages"


def test_noalloc_multi_plan_two_calls():
    _need_gpu()
    import torch

    inp = uneven_inputs(3300, 3000)
    plans = [gpu_plan(c) for c in inp["codes"]]
    llr = torch.from_numpy(inp["raw"]).cuda()
    for n in (3000, 700):
        print(f"multi-plan int16, {len(plans)} plans, {n} frames", flush=True)
        fr = torch.from_numpy(np.ascontiguousarray(inp["desc"][:n]).view(np.int32)).cuda()
        _assert_same(_both(plans, llr, frames=fr), f"multi-plan, {n} frames")


def test_noalloc_plain_float_two_calls():
    _need_gpu()
    import torch
    from paper_1710_08314_amd import polar as P

    import oracle as O
    from tests.gpu_util import make_inputs, oracle_code

    fz = O.construct(256, 128, 0, 8, 2.0)
    code = oracle_code(256, 128, 8, 0x07, fz, quant="f32", algo="ca", L=4)
    plan = gpu_plan(code)
    for n in (1000, 257):
        print(f"plain float32 CA-SCL L = 4, {n} frames", flush=True)
        _, llr = make_inputs(code, n, 40 + n, 2.5)
        t = torch.from_numpy(np.ascontiguousarray(llr)).cuda()
        _assert_same(_both(plan, t, schedule=1), f"plain float32, {n} frames")


def test_noalloc_rejects_oversized_batch():
    _need_gpu()
    import torch
    from paper_1710_08314_amd import polar as P

    plan = P.Plan(256, 128, 8, 0x07, design_ebn0_db=2.0, algo=P.CA_SCL, L=4, quant=P.I8)
    n = (1 << 21) + 1  # one frame above the limit: rejected before any device work
    llr = torch.zeros((1, 256), dtype=torch.int8, device="cuda")
    info = torch.zeros((1, 4), dtype=torch.int32, device="cuda")
    status = torch.zeros((1, 8), dtype=torch.uint8, device="cuda")
    with pytest.raises(P.PolarError) as e:
        P.decode_batch_noalloc(plan, llr, info, status, n_frames=n)
    assert e.value.code == -7
