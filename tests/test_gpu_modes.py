"""GPU parity (through the C ABI) of the modes and edge cases beside the default
path: the alpha variants of Eq. 13, the paper's literal full-support windows,
uncropped packets of every frame-count class of the uneven stream, an all-zero
packet, the Jacobi sweep cap, caller-given weights in a batched call, and calls
made while the caller captures the stream."""
import multiprocessing as mp

import numpy as np
import pytest

import oracle as O
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


# ------------------------------------------------------------------ Eq. 13 variants

@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("mode", [1, 2])
def test_pd_modes(lcf, ctx, mode, prec):
    """alpha_d = 1 (PD_SUM) and Eq. 13 divided by sum_d alpha_d w_d^2
    (PD_EQ13_COMPENSATED) on a clinical packet, both precisions."""
    iq, mask = synth.make_packet(synth.spec_clinical(4))
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID, pd_mode=mode)
    tol = 1e-5 if prec == lcf.PREC_FP32 else 1e-3
    check_end_to_end(lcf, ctx, iq, mask, 8, 8, thr, tol, 0.1, f"pd_mode={mode} prec={prec}", precision=prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_full_support_windows(lcf, ctx, prec):
    """trunc_sigmas = 0: every window spans the whole image (the paper's literal
    Eq. 11), so each subset's covariance runs over all 49,152 pixels."""
    iq, mask = synth.make_packet(synth.spec_clinical(5))
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
    tol = 1e-5 if prec == lcf.PREC_FP32 else 1e-3
    check_end_to_end(lcf, ctx, iq, mask, 8, 8, thr, tol, 0.1, f"full-support windows prec={prec}",
                     precision=prec, trunc_sigmas=0.0)


# ------------------------------------------------------------------ uneven stream, uncropped

def _gen(spec):
    return synth.make_packet(spec)


@pytest.mark.parametrize("prec", [0, 1])
def test_stream_classes_uncropped_vs_oracle(lcf, ctx, prec):
    """The first packet of each frame-count class (32, 64, 100, 200) of the
    uneven stream at its full size, filtered together in one batched call; each
    equals its single call bitwise and matches the oracle."""
    lst = synth.batch_specs(3000, 16)
    picks, seen = [], set()
    for i, (spec, g) in enumerate(lst):
        if spec.nt not in seen:
            seen.add(spec.nt)
            picks.append(i)
    assert sorted(seen) == [32, 64, 100, 200]
    with mp.get_context("spawn").Pool(4) as pool:       # workers run numpy only
        data = pool.map(_gen, [lst[i][0] for i in picks])
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
    dev = [torch.from_numpy(iq).cuda() for iq, _ in data]
    grids = [(lst[i][1], lst[i][1]) for i in picks]
    say(f"[stream classes prec={prec}] " + ", ".join(f"{tuple(d.shape)} g={g[0]}" for d, g in zip(dev, grids)))
    ios, pds = ctx.filter_batch(dev, grids, thr, precision=prec, iq_out=True)
    torch.cuda.synchronize()
    assert ctx.sync() == 0
    tol = 1e-5 if prec == lcf.PREC_FP32 else 1e-3
    for k, i in enumerate(picks):
        _, _, io1, pd1 = check_end_to_end(lcf, ctx, data[k][0], data[k][1], grids[k][0], grids[k][1], thr, tol,
                                          0.1, f"stream packet {i}", precision=prec)
        assert np.array_equal(ios[k].cpu().numpy(), io1) and np.array_equal(pds[k].cpu().numpy(), pd1), k


# ------------------------------------------------------------------ degenerate cases

@pytest.mark.parametrize("prec", [0, 1])
def test_zero_packet(lcf, ctx, prec):
    """An all-zero packet: R = 0, every eigenvalue 0, the curvature rule flags
    the subset (lambda_1 <= 0) and keeps every component (k = 0), alpha = 0, and
    the filtered IQ and power Doppler are exactly zero."""
    say(f"[zero packet prec={prec}]")
    iq = np.zeros((32, 48, 40), dtype=np.complex64)
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_HARD)
    io, pd, dg = ctx.filter(torch.from_numpy(iq).cuda(), 2, 2, thr, precision=prec, diag=True)
    torch.cuda.synchronize()
    assert ctx.sync() == 0
    d = {k: v.cpu().numpy() for k, v in dg.items()}
    res = O.filter_packet(iq, 2, 2, O.Threshold(cut=O.CUT_KNEE, shape=O.SHAPE_HARD))
    assert np.all(d["flags"] & lcf.FLAG_NONPOSITIVE)
    assert np.all(res["flags"]) and res["k"] == [0, 0, 0, 0]
    assert np.array_equal(d["k"], np.zeros(4, dtype=np.int32))
    assert np.array_equal(d["weights"], np.ones((4, 32), dtype=np.float32))
    assert np.array_equal(d["eigvals"], np.zeros((4, 32)))
    assert np.array_equal(d["alpha"], np.zeros(4)) and res["alpha"] == [0.0] * 4
    assert np.array_equal(io.cpu().numpy(), np.zeros_like(iq))
    assert np.array_equal(pd.cpu().numpy(), np.zeros((48, 40), dtype=np.float32))


def test_jacobi_sweep_cap_reported(lcf, ctx):
    """The Jacobi solver stopped at a cap of one sweep flags every subset and
    lcf_sync returns LCF_ERR_NO_CONVERGENCE once; the next call is clean."""
    say("[sweep cap]")
    iq, _ = synth.make_packet(synth.spec_small(10))
    thr = lcf.Threshold(cut=lcf.CUT_KNEE)
    dev = torch.from_numpy(iq).cuda()
    ctx.set_option(lcf.OPT_EVD, lcf.EVD_JACOBI)
    ctx.set_option(lcf.OPT_MAX_SWEEPS, 1)
    try:
        _, _, dg = ctx.filter(dev, 3, 3, thr, diag=True)
        torch.cuda.synchronize()
        flags = dg["flags"].cpu().numpy()
        assert np.all(flags & lcf.FLAG_NO_CONVERGE)
        assert ctx.sync() == 6                         # LCF_ERR_NO_CONVERGENCE
        assert ctx.sync() == 0
    finally:
        ctx.set_option(lcf.OPT_MAX_SWEEPS, 30)
        ctx.set_option(lcf.OPT_EVD, lcf.EVD_TRIDIAGONAL)
    _, _, dg = ctx.filter(dev, 3, 3, thr, diag=True)
    torch.cuda.synchronize()
    assert ctx.sync() == 0
    assert not np.any(dg["flags"].cpu().numpy() & lcf.FLAG_NO_CONVERGE)


# ------------------------------------------------------------------ boundary

def test_batch_explicit_weights_match_single(lcf, ctx):
    """Caller-given weights in a batched call (packets' [nd][nt] blocks back to
    back) equal the single calls, with packets of two frame-count classes."""
    say("[batch explicit weights]")
    specs = [synth.PacketSpec(64, 48, 32, 50.0, 0.3, ((20, 3, 0.5),), seed=31),
             synth.PacketSpec(56, 40, 80, 50.0, 0.4, ((25, 3, 0.5),), seed=32),
             synth.PacketSpec(48, 56, 32, 45.0, 0.6, ((30, 4, 0.9),), seed=33)]
    grids = [(2, 2), (3, 3), (2, 3)]
    rng = np.random.default_rng(34)
    iqs = [torch.from_numpy(synth.make_packet(s)[0]).cuda() for s in specs]
    ews = [torch.from_numpy(rng.uniform(0.0, 1.0, size=(g[0] * g[1], s.nt)).astype(np.float32))
           for s, g in zip(specs, grids)]
    thr = lcf.Threshold(cut=lcf.CUT_EXPLICIT)
    ios, pds = ctx.filter_batch(iqs, grids, thr, iq_out=True, explicit_w=ews)
    for i in range(3):
        io1, pd1, _ = ctx.filter(iqs[i], grids[i][0], grids[i][1], thr, explicit_w=ews[i])
        torch.cuda.synchronize()
        assert torch.equal(ios[i], io1) and torch.equal(pds[i], pd1), i
    assert ctx.sync() == 0


def test_calls_under_caller_capture_are_refused(lcf, ctx):
    """Entry points that stage plans or grow buffers return LCF_ERR_UNSUPPORTED
    while the caller captures the stream, before launching anything."""
    say("[capture refused]")
    iq = torch.from_numpy(synth.make_packet(synth.spec_small(11))[0]).cuda()
    out = (torch.empty_like(iq), torch.empty((64, 64), dtype=torch.float32, device="cuda"))
    a = torch.eye(8, dtype=torch.complex128, device="cuda").reshape(1, 8, 8).contiguous()
    thr = lcf.Threshold(cut=lcf.CUT_KNEE)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    codes = []
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        g.capture_begin()
        try:
            for call in (lambda: ctx.filter(iq, 3, 3, thr, out=out),
                         lambda: ctx.filter_batch([iq], [(3, 3)], thr, outs=[out]),
                         lambda: ctx.heevd(a)):
                try:
                    call()
                    codes.append(0)
                except lcf.LcfError as e:
                    codes.append(e.status)
        finally:
            g.capture_end()
    torch.cuda.synchronize()
    assert codes == [2, 2, 2], codes
    # the same calls work outside capture
    ctx.filter(iq, 3, 3, thr, out=out)
    torch.cuda.synchronize()
    assert ctx.sync() == 0
