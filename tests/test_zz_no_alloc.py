"""GPU test of the allocation-free entry point lcf_filter_noalloc: the same
packets through it and through lcf_filter (its arena twin) give the same
filtered IQ, power Doppler and per-subset decisions; two calls in a row, the
second with a smaller packet (the fixed block keeps the first call's contents);
a call whose workspace exceeds the fixed block is refused before any launch."""
import os

import numpy as np
import pytest

import synth
from parity import say, rel_fro, pd_db_error

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CKPT = os.path.join(ROOT, "paper_2405_11105_amd", "weights", "mlp_512x256x128.ckpt")


@pytest.fixture(scope="module")
def ctx(lcf):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    c = lcf.Context(0)
    yield c
    c.close()


def _outs(iq):
    nt, ny, nx = iq.shape
    return (torch.empty_like(iq), torch.empty((ny, nx), dtype=torch.float32, device=iq.device))


def _both(lcf, ctx, iq_np, mask, gy, gx, thr, prec, tol_fro, name):
    """One call through each entry point on the same packet; compare outputs and
    the per-subset integer decisions."""
    say(f"[noalloc {name}] shape={iq_np.shape} grid={gy}x{gx} cut={thr.cut} prec={prec}")
    iq = torch.from_numpy(iq_np).cuda()
    # fresh outputs, poisoned, so a missing write shows
    oa = _outs(iq)
    oa[0].fill_(float("nan"))
    oa[1].fill_(float("nan"))
    ioa, pda, da = ctx.filter(iq, gy, gx, thr, precision=prec, diag=True, out=oa, noalloc=True)
    torch.cuda.synchronize()
    assert ctx.sync() == 0
    ob = _outs(iq)
    iob, pdb, db = ctx.filter(iq, gy, gx, thr, precision=prec, diag=True, out=ob)
    torch.cuda.synchronize()
    assert ctx.sync() == 0
    ioa, pda, iob, pdb = (t.cpu().numpy() for t in (ioa, pda, iob, pdb))
    assert np.all(np.isfinite(ioa)) and np.all(np.isfinite(pda))
    e_fro = rel_fro(ioa, iob)
    emax, e99, _, npx = pd_db_error(pda, pdb, mask)
    same = bool(np.array_equal(ioa, iob) and np.array_equal(pda, pdb))
    say(f"   vs lcf_filter: rel_fro={e_fro:.3e} pd_db max={emax:.2e} p99={e99:.2e} n={npx} bitwise={same}")
    for key in ("k", "flags", "rank"):
        assert np.array_equal(da[key].cpu().numpy(), db[key].cpu().numpy()), key
    assert e_fro <= tol_fro
    assert emax <= 0.1


def test_noalloc_matches_arena_entry_point(lcf, ctx):
    """Clinical packet (256 x 192 x 128, 8 x 8 windows: 151 MiB of workspace,
    the largest of the parity workloads that fits), then a smaller one in the
    other precision, then the learned weights on a clinical packet."""
    iq, mask = synth.make_packet(synth.spec_clinical(7))
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
    _both(lcf, ctx, iq, mask, 8, 8, thr, lcf.PREC_FP32, 1e-5, "clinical fp32")
    iq, mask = synth.make_packet(synth.spec_small(0))
    thr = lcf.Threshold(cut=lcf.CUT_FIXED_K, k_fixed=4)
    _both(lcf, ctx, iq, mask, 3, 3, thr, lcf.PREC_BF16X3, 1e-3, "small bf16x3")
    ctx.mlp_load(CKPT)
    iq, mask = synth.make_packet(synth.spec_clinical(8))
    thr = lcf.Threshold(cut=lcf.CUT_MLP, shape=lcf.SHAPE_SIGMOID)
    _both(lcf, ctx, iq, mask, 8, 8, thr, lcf.PREC_BF16X3, 1e-3, "clinical mlp bf16x3")


def test_noalloc_refuses_oversized_workspace(lcf, ctx):
    """512 x 256 x 128 with 16 x 16 windows needs about 546 MiB of workspace:
    refused with LCF_ERR_SCRATCH_LIMIT, outputs untouched."""
    iq = torch.zeros((128, 512, 256), dtype=torch.complex64, device="cuda")
    io, pd = _outs(iq)
    pd.fill_(-1.0)
    thr = lcf.Threshold(cut=lcf.CUT_FIXED_K, k_fixed=4)
    with pytest.raises(lcf.LcfError) as ei:
        ctx.filter(iq, 16, 16, thr, out=(io, pd), noalloc=True)
    assert ei.value.status == 8
    torch.cuda.synchronize()
    assert ctx.sync() == 0
    assert bool(torch.all(pd == -1.0))
