"""GPU parity (through the C ABI) of sliding packets (lcf_stream_*): a recording
is filtered as packets that slide by `hop` frames, the covariance carried
from push to push; every push is compared with the oracle filtering that
packet from scratch, and with lcf_filter on the same packet."""
import pytest

import synth
from parity import say, compare_with_oracle, rel_fro, pd_db_error

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx(lcf):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    c = lcf.Context(0)
    yield c
    c.close()


def _recording(ny, nx, nt, hop, pushes, seed, tissue_db=50.0):
    spec = synth.PacketSpec(ny, nx, nt + (pushes - 1) * hop, tissue_db, 0.6,
                            ((ny // 4, 3, 0.3), (ny // 2, 5, 0.8), (3 * ny // 4, 2, 0.1)), seed=seed)
    return synth.make_packet(spec)


def _run(lcf, ctx, ny, nx, nt, gy, gx, hop, pushes, thr, prec, seed, tol, name):
    rec, mask = _recording(ny, nx, nt, hop, pushes, seed)
    rec_t = torch.from_numpy(rec).cuda()
    sm = lcf.Stream(ctx, ny, nx, nt, gy, gx, thr, precision=prec)
    try:
        for p in range(pushes):
            pk = rec_t[p * hop:p * hop + nt]          # frame-major: a contiguous view
            assert pk.is_contiguous()
            say(f"[{name}] push {p} hop={hop} frames {p * hop}..{p * hop + nt - 1}")
            io, pd, d = sm.push(pk, hop, diag=True)
            torch.cuda.synchronize()
            assert ctx.sync() == 0
            d = {k: v.cpu().numpy() for k, v in d.items()}
            io, pd = io.cpu().numpy(), pd.cpu().numpy()
            compare_with_oracle(lcf, rec[p * hop:p * hop + nt], mask, gy, gx, thr, io, pd, d, tol, 0.1)
            # the packet through the two Gram passes instead
            io2, pd2, _ = ctx.filter(pk, gy, gx, thr, precision=prec)
            torch.cuda.synchronize()
            e = rel_fro(io, io2.cpu().numpy())
            emax, _, _, _ = pd_db_error(pd, pd2.cpu().numpy(), mask)
            say(f"   vs lcf_filter: rel_fro={e:.2e} pd_db max={emax:.2e}")
            assert e <= 2 * tol and emax <= 0.1
    finally:
        sm.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_sliding_stream_vs_oracle(lcf, ctx, prec):
    """9 pushes of 128 x 96 x 64 packets sliding by 5 frames, 4 x 4 windows,
    curvature rule with sigmoid weights."""
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
    _run(lcf, ctx, 128, 96, 64, 4, 4, 5, 9, thr, prec, 31, 1e-5 if prec == 0 else 1e-3, f"slide prec={prec}")


@pytest.mark.parametrize("hop", [1, 20])
def test_sliding_stream_hop_sizes(lcf, ctx, hop):
    """A one-frame hop and a hop of more than one group of 16 new columns."""
    thr = lcf.Threshold(cut=lcf.CUT_FIXED_K, k_fixed=3)
    _run(lcf, ctx, 80, 72, 48, 3, 3, hop, 4, thr, 0, 40 + hop, 1e-5, f"slide hop={hop}")


def test_sliding_stream_clinical(lcf, ctx):
    """Clinical shape (256 x 192 x 128, 8 x 8 windows), split BF16, 3 pushes."""
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
    _run(lcf, ctx, 256, 192, 128, 8, 8, 5, 3, thr, 1, 51, 1e-3, "slide clinical bf16x3")


def test_stream_argument_errors(lcf, ctx):
    thr = lcf.Threshold(cut=lcf.CUT_FIXED_K, k_fixed=3)
    sm = lcf.Stream(ctx, 32, 32, 16, 2, 2, thr)
    try:
        iq = torch.zeros((16, 32, 32), dtype=torch.complex64, device="cuda")
        for hop in (0, 17):
            with pytest.raises(lcf.LcfError) as ei:
                sm.push(iq, hop)
            assert ei.value.status == 1
    finally:
        sm.close()
    with pytest.raises(lcf.LcfError):
        lcf.Stream(ctx, 32, 32, 300, 2, 2, thr)
