"""Batched uneven decoding: frames of thousands of different codes and
decoders in one call (per frame N in {128 .. 2048}, rate in {1/4 .. 5/6},
L in {2, 8, 32}, 20% shortened, CRC-11, int16, Eb/N0 ~ U[1, 4] dB), decoded
by the class schedule with autotuned kernel choices; HIP-graph capture and
replay of a decode.

Parity: sampled frames element by element against the oracle (bit-exact in
int16), every frame's list size and live paths, and frames decoded alone
equal to the same frames decoded in the mix."""
import numpy as np
import pytest

from tests.gpu_util import check_uneven, gpu_plan, uneven_inputs

pytestmark = pytest.mark.gpu

N_FRAMES = 1 << 16


@pytest.fixture(scope="module")
def uneven():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    inp = uneven_inputs(3100, N_FRAMES)
    print(f"{N_FRAMES} frames, {len(inp['specs'])} plans", flush=True)
    plans = [gpu_plan(c) for c in inp["codes"]]
    llr = torch.from_numpy(inp["raw"]).cuda()
    fr = torch.from_numpy(inp["desc"].view(np.int32)).cuda()
    return inp, plans, llr, fr


def test_uneven_batch_autotuned(uneven):
    import torch
    from paper_1710_08314_amd import polar as P

    inp, plans, llr, fr = uneven
    info, status, pml = P.decode_batch(plans, llr, frames=fr, with_pm_lists=True, autotune=True)
    torch.cuda.synchronize()
    desc = P.schedule_describe(plans)
    print(desc, flush=True)
    assert "tuned=1" in desc
    info_h = info.cpu().numpy().view(np.uint32)
    st_h = status.cpu().numpy()
    pml_h = pml.cpu().numpy().view(np.uint32)
    rng = np.random.default_rng(7)
    sample = np.sort(rng.choice(N_FRAMES, 1500, replace=False))
    check_uneven(inp, info_h, st_h, sample, pml_h)
    # every frame ran its plan's single stage
    Ls = np.array([s[2] for s in inp["specs"]])[inp["plan_of"]]
    st = P.status_fields(st_h)
    assert np.array_equal(st["L_used"], Ls)
    assert (st["n_paths"] <= Ls).all() and (st["n_paths"] >= 1).all()
    # a second call uses the cached choice and gives the same outputs
    info2, status2, _ = P.decode_batch(plans, llr, frames=fr, autotune=True)
    torch.cuda.synchronize()
    assert np.array_equal(info2.cpu().numpy(), info.cpu().numpy())
    assert np.array_equal(status2.cpu().numpy(), st_h)


def test_alone_equals_in_mix(uneven):
    """Frames of three plans decoded as single-plan batches (tiered schedule)
    equal the same frames decoded inside the uneven batch."""
    import torch
    from paper_1710_08314_amd import polar as P

    inp, plans, llr, fr = uneven
    info, status, _ = P.decode_batch(plans, llr, frames=fr)
    torch.cuda.synchronize()
    info_h = info.cpu().numpy().view(np.uint32)
    st_h = status.cpu().numpy()
    counts = np.bincount(inp["plan_of"], minlength=len(plans))
    es = 2
    for pi in np.argsort(-counts)[:3]:
        fs = np.nonzero(inp["plan_of"] == pi)[0]
        cd = inp["codes"][pi]
        alone = np.stack([inp["raw"][inp["desc"][f, 0]:inp["desc"][f, 0] + cd.n_tx * es]
                          .view(np.int16) for f in fs])
        a_info, a_st, _ = P.decode_batch(plans[pi], torch.from_numpy(alone).cuda())
        torch.cuda.synchronize()
        a_info = a_info.cpu().numpy().view(np.uint32)
        iw = (cd.k_data + 31) // 32
        for j, f in enumerate(fs):
            o = inp["out_off"][f]
            assert np.array_equal(a_info[j, :iw], info_h[o:o + iw]), f"plan {pi} frame {f}"
        assert np.array_equal(a_st.cpu().numpy(), st_h[fs])


def test_graph_replay_uneven(uneven):
    """A captured decode replayed three times, with eager work and new input
    contents between replays: every replay equals the eager decode of what
    the buffers held."""
    import torch
    from paper_1710_08314_amd import polar as P

    inp, plans, llr, fr = uneven
    work = llr.clone()
    g = P.Graph(plans, work, frames=fr, with_pm_lists=True)
    ref = P.decode_batch(plans, work, frames=fr, with_pm_lists=True)
    alt = torch.flip(llr.view(torch.int16), dims=[0]).view(torch.uint8).contiguous()
    ref_alt = P.decode_batch(plans, alt, frames=fr, with_pm_lists=True)
    torch.cuda.synchronize()
    for rep in range(3):
        src, want = (llr, ref) if rep != 1 else (alt, ref_alt)
        work.copy_(src)
        g.info.zero_()
        g.status.zero_()
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for a, b in zip((g.info, g.status, g.pm_lists), want):
            assert torch.equal(a, b), f"replay {rep}"
        # eager work between replays
        P.decode_batch(plans, alt, frames=fr)
        torch.cuda.synchronize()
    g.close()


def test_graph_replay_adaptive_single_plan():
    """Graph capture of the tiered schedule (per-frame state words, and the
    frame list of the frame-per-lane L = 2 stage) on the (1024, 488 +
    CRC-24) code with FA L = 1 -> 8, int8."""
    import torch

    import oracle as O
    from paper_1710_08314_amd import polar as P
    from tests.gpu_util import make_inputs, oracle_code

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fz = O.construct(1024, 512, 0, 24, 2.5)
    code = oracle_code(1024, 512, 24, 0x1864CFB, fz, quant="i8", algo="fa", L_max=8)
    plan = gpu_plan(code)
    _, llr_a = make_inputs(code, 3000, 11, 2.0)
    _, llr_b = make_inputs(code, 3000, 12, 2.5)
    a, b = torch.from_numpy(llr_a).cuda(), torch.from_numpy(llr_b).cuda()
    work = a.clone()
    g = P.Graph(plan, work, with_pm_lists=True)
    refs = [P.decode_batch(plan, x, with_pm_lists=True) for x in (a, b)]
    torch.cuda.synchronize()
    for rep, k in enumerate((0, 1, 0, 1)):
        work.copy_((a, b)[k])
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for x, y in zip((g.info, g.status, g.pm_lists), refs[k]):
            assert torch.equal(x, y), f"replay {rep}"
        P.decode_batch(plan, b)  # eager work between replays
        torch.cuda.synchronize()
    # the replays are the oracle's decodes too (sampled)
    ref = O.decode(code, llr_b[:200])
    st = P.status_fields(g.status.cpu().numpy()[:200])
    assert np.array_equal(st["L_used"], ref.L_used)
    assert np.array_equal(P.unpack_bits(g.info.cpu().numpy().view(np.uint32)[:200], code.k_data),
                          ref.info)
    g.close()


def test_mixed_quantisations_one_decode():
    """Plans of float32, int16 and int8 LLRs (CA-SCL, N in {128, 256, 512},
    L in {2, 8}, CRC-11) in one decode call: the class schedule splits the
    frames by LLR type too.  Every frame is checked against the oracle
    (int: bit-exact bits, metric, metric list; float32: metrics within 1e-4,
    bits equal unless near-tie, flags equal), and against the frames of each
    type decoded alone."""
    import torch

    import oracle as O
    from paper_1710_08314_amd import polar as P
    from paper_1710_08314_amd import synth
    from tests.gpu_util import PM_RTOL, QMAP, oracle_code, pack_inputs, pm_values

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c, poly = synth.C3_CRC
    specs = [(N, K, L, q) for q in ("f32", "i16", "i8") for (N, K) in ((128, 48), (256, 140), (512, 300))
             for L in (2, 8)]
    codes = [oracle_code(N, K, c, poly, O.construct(N, K, 0, c, synth.C3_DESIGN_DB), quant=q,
                         algo="ca", L=L) for (N, K, L, q) in specs]
    rng = np.random.default_rng(3400)
    n = 1800
    plan_of = rng.integers(0, len(specs), n)
    ebn0 = rng.uniform(1.0, 3.0, n)
    inp = pack_inputs(codes, plan_of, ebn0, 3401)
    plans = [gpu_plan(cd) for cd in codes]
    llr = torch.from_numpy(inp["raw"]).cuda()
    fr = torch.from_numpy(inp["desc"].view(np.int32)).cuda()
    info, status, pml = P.decode_batch(plans, llr, frames=fr, with_pm_lists=True)
    torch.cuda.synchronize()
    desc = P.schedule_describe(plans)
    print(desc, flush=True)
    assert " q0 " in desc and " q1 " in desc and " q2 " in desc
    info_h = info.cpu().numpy().view(np.uint32)
    st = P.status_fields(status.cpu().numpy())
    pml_h = pml.cpu().numpy().view(np.uint32)
    for pi, cd in enumerate(codes):
        fs = np.nonzero(plan_of == pi)[0]
        if not len(fs):
            continue
        es = np.dtype(O.DTYPES[cd.quant]).itemsize
        llrs = np.stack([inp["raw"][inp["desc"][f, 0]:inp["desc"][f, 0] + cd.n_tx * es]
                         .view(O.DTYPES[cd.quant]) for f in fs])
        ref = O.decode(cd, llrs, threads=8)
        iw = (cd.k_data + 31) // 32
        bits = np.stack([P.unpack_bits(info_h[inp["out_off"][f]:inp["out_off"][f] + iw], cd.k_data)
                         for f in fs])
        assert np.array_equal(st["L_used"][fs], ref.L_used), specs[pi]
        assert np.array_equal(st["crc_ok"][fs], ref.crc_ok), specs[pi]
        assert np.array_equal(st["n_paths"][fs], ref.n_pm), specs[pi]
        assert np.array_equal(st["near_tie"][fs], ref.near_tie), specs[pi]
        g_pm = pm_values(st["pm_bits"][fs], cd.quant)
        if cd.quant == O.F32:
            assert (np.abs(g_pm - ref.pm) <= PM_RTOL * np.maximum(1.0, np.abs(ref.pm))).all(), specs[pi]
            eq = (bits == ref.info).all(axis=1)
            assert (eq | (ref.near_tie == 1)).all(), specs[pi]
        else:
            assert np.array_equal(g_pm, ref.pm), specs[pi]
            assert np.array_equal(bits, ref.info), specs[pi]
            for j, f in enumerate(fs):
                k = int(ref.n_pm[j])
                assert np.array_equal(pml_h[f, :k].view(np.int32), ref.pm_list[j, :k].astype(np.int32))
    # each type decoded alone (its own plans only) gives the same outputs
    for q in ("f32", "i16", "i8"):
        sub = [i for i, s in enumerate(specs) if s[3] == q]
        fs = np.nonzero(np.isin(plan_of, sub))[0]
        remap = {p: j for j, p in enumerate(sub)}
        d = inp["desc"][fs].copy()
        d[:, 3] = [remap[int(p)] for p in d[:, 3]]
        a_info, a_st, _ = P.decode_batch([plans[i] for i in sub], llr,
                                         frames=torch.from_numpy(d.view(np.int32)).cuda())
        torch.cuda.synchronize()
        a_info_h = a_info.cpu().numpy().view(np.uint32)
        assert np.array_equal(a_st.cpu().numpy(), status.cpu().numpy()[fs]), q
        for f in fs:
            o = inp["out_off"][f]
            iw = (codes[plan_of[f]].k_data + 31) // 32
            assert np.array_equal(a_info_h[o:o + iw], info_h[o:o + iw]), (q, f)
