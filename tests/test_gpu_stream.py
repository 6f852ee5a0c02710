"""The uneven packet stream (Nt in {32, 64, 100, 200}, images 128..400 x
128..256, square window grids 2..10) filtered in one batched call: parity of
cropped packets against the FP64 oracle, and the full-size stream against
per-packet calls."""
import multiprocessing as mp

import numpy as np
import pytest

import synth
from parity import say, check_end_to_end

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx(lcf):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    c = lcf.Context(0)
    yield c
    c.close()


def _gen(spec):
    return synth.make_packet(spec)


def _packets(n):
    lst = synth.batch_specs(3000, n)
    with mp.get_context("spawn").Pool(8) as pool:      # workers run numpy only
        data = pool.map(_gen, [s for s, _ in lst])
    return lst, data


def test_stream_cropped_batched_vs_oracle(lcf, ctx):
    """One packet of each Nt class, cropped to at most 112 x 96 pixels, filtered
    together in one call; each must equal its single call bitwise and match the
    oracle (knee + sigmoid rule, FP32 path)."""
    lst, data = _packets(8)
    picks, seen = [], set()
    for i, (spec, g) in enumerate(lst):
        if spec.nt not in seen:
            seen.add(spec.nt)
            picks.append(i)
    assert sorted(seen) == [32, 64, 100, 200]
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
    iqs, masks, grids = [], [], []
    for i in picks:
        iq, mask = data[i]
        iqs.append(np.ascontiguousarray(iq[:, :112, :96]))
        masks.append(mask[:112, :96])
        g = lst[i][1]
        grids.append((g, g))
    dev = [torch.from_numpy(x).cuda() for x in iqs]
    ios, pds = ctx.filter_batch(dev, grids, thr, iq_out=True)
    torch.cuda.synchronize()
    assert ctx.sync() == 0
    for k, i in enumerate(picks):
        io1, pd1, _ = ctx.filter(dev[k], grids[k][0], grids[k][1], thr)
        torch.cuda.synchronize()
        assert torch.equal(ios[k], io1) and torch.equal(pds[k], pd1), k
        check_end_to_end(lcf, ctx, iqs[k], masks[k], grids[k][0], grids[k][1], thr, 1e-5, 0.1,
                         f"stream packet {i} nt={iqs[k].shape[0]} g={grids[k][0]}")


def test_stream_full_size_one_call(lcf, ctx):
    """Sixteen full-size packets of the stream in one batched call (split-BF16):
    no device-side flags, and sampled packets equal their single calls."""
    lst, data = _packets(16)
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
    dev = [torch.from_numpy(iq).cuda() for iq, _ in data]
    grids = [(g, g) for _, g in lst]
    say(f"[full stream] {len(dev)} packets, nt {sorted(set(s.nt for s, _ in lst))}, "
        f"subsets {sum(g * g for _, g in lst)}")
    ios, pds = ctx.filter_batch(dev, grids, thr, precision=lcf.PREC_BF16X3, iq_out=True)
    torch.cuda.synchronize()
    assert ctx.sync() == 0
    for k in (0, 5, 11):
        io1, pd1, _ = ctx.filter(dev[k], grids[k][0], grids[k][1], thr, precision=lcf.PREC_BF16X3)
        torch.cuda.synchronize()
        assert torch.equal(ios[k], io1) and torch.equal(pds[k], pd1), k
        assert torch.isfinite(pds[k]).all()


def test_autotune_choice_roundtrip(lcf, ctx, tmp_path):
    """Autotuned plans give the same filter (the tile height does not change the
    arithmetic; the split-K chunk only moves FP32 rounding), and the stored
    choices reproduce the tuned run bitwise in a fresh context."""
    iq, mask = synth.make_packet(synth.spec_clinical(3))
    dev = torch.from_numpy(iq).cuda()
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
    io0, pd0, _ = ctx.filter(dev, 8, 8, thr)
    tuned = lcf.Context(0, autotune=1)
    try:
        io1, pd1, _ = tuned.filter(dev, 8, 8, thr)
        torch.cuda.synchronize()
        assert tuned.sync() == 0
        path = str(tmp_path / "tune.txt")
        tuned.tune_save(path)
        lines = open(path).read().split("\n")
        say(f"[autotune] {lines[0]}")
        assert len([x for x in lines if x.strip()]) == 1 and len(lines[0].split()) == 5
        e_io = float(torch.linalg.vector_norm(io1 - io0) / torch.linalg.vector_norm(io0))
        e_pd = float(torch.max(torch.abs(pd1 - pd0) / pd0))
        assert e_io <= 1e-5 and e_pd <= 1e-4, (e_io, e_pd)
        again = lcf.Context(0)
        try:
            again.tune_load(path)
            io2, pd2, _ = again.filter(dev, 8, 8, thr)
            torch.cuda.synchronize()
            assert torch.equal(io1, io2) and torch.equal(pd1, pd2)
            bad = tmp_path / "bad.txt"
            bad.write_text("ntp128_p0_s0_S6_N13 1024\n")
            with pytest.raises(lcf.LcfError) as ei:
                again.tune_load(str(bad))
            assert ei.value.status == 1
        finally:
            again.close()
    finally:
        tuned.close()


def test_stream_64_packets_one_graph_call(lcf, ctx):
    """All 64 packets of the uneven stream in one batched call, captured into a
    hipGraph and replayed (split BF16): replays are bitwise equal, one packet
    per Nt class equals its single call bitwise, and the autotuned plan of the
    same call agrees to FP32 rounding (it only moves the split-K chunks)."""
    lst, data = _packets(64)
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
    grids = [(g, g) for _, g in lst]
    say(f"[64-packet stream] nt {sorted(set(s.nt for s, _ in lst))}, subsets {sum(g * g for _, g in lst)}")
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        dev = [torch.from_numpy(iq).cuda() for iq, _ in data]
        del data
        outs = [(torch.empty_like(d), torch.empty(d.shape[1:], dtype=torch.float32, device="cuda")) for d in dev]
        g = lcf.Context(0, use_graph=1)
        t = lcf.Context(0, use_graph=1, autotune=1)
        try:
            g.filter_batch(dev, grids, thr, precision=lcf.PREC_BF16X3, outs=outs)        # capture
            st.synchronize()
            first = [(io.clone(), pd.clone()) for io, pd in outs]
            g.filter_batch(dev, grids, thr, precision=lcf.PREC_BF16X3, outs=outs)        # replay
            st.synchronize()
            assert g.sync() == 0
            for (a, b), (c, d) in zip(first, outs):
                assert torch.equal(a, c) and torch.equal(b, d)
            picks = {}
            for k, (s, _) in enumerate(lst):
                picks.setdefault(s.nt, k)
            for nt, k in sorted(picks.items()):
                io1, pd1, _ = ctx.filter(dev[k], grids[k][0], grids[k][1], thr, precision=lcf.PREC_BF16X3)
                st.synchronize()
                assert torch.equal(first[k][0], io1) and torch.equal(first[k][1], pd1), (nt, k)
            ios_t, pds_t = t.filter_batch(dev, grids, thr, precision=lcf.PREC_BF16X3, iq_out=True)
            st.synchronize()
            assert t.sync() == 0
            worst_io = max(float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
                           for a, (b, _) in zip(ios_t, first))
            worst_pd = max(float(torch.max(torch.abs(a - b) / b)) for a, (_, b) in zip(pds_t, first))
            say(f"   autotuned vs default plan: iq {worst_io:.2e}, pd {worst_pd:.2e}")
            assert worst_io <= 1e-4 and worst_pd <= 1e-3
        finally:
            g.close()
            t.close()
