"""GPU parity of the learned-weight kernels (forward, backward, Adam, checkpoint)
against the FP64 oracle, and their use inside the filter."""
import os
import sys
import tempfile

import numpy as np
import pytest

import oracle as O
from oracle import mlp as M
import synth
from parity import rel_fro, pd_db_error

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(lcf):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    c = lcf.Context(0)
    yield c
    c.close()


def _spectra(b, seed):
    rng = np.random.default_rng(seed)
    lam = np.sort(10.0 ** rng.uniform(-7.5, 0, size=(b, M.NT)), axis=1)[:, ::-1] * 10.0 ** rng.uniform(4, 9, size=(b, 1))
    k = rng.integers(3, 12, size=(b, 1))
    t = 1.0 / (1.0 + np.exp(-2.0 * (np.arange(1, M.NT + 1)[None, :] - k)))
    return np.ascontiguousarray(lam), np.ascontiguousarray(t.astype(np.float32))


def test_forward_matches_oracle(lcf, ctx):
    _say("[mlp forward parity]")
    ctx.mlp_init(7)
    p = M.unflatten(ctx.mlp_get_params())
    lam, _ = _spectra(300, 1)
    w_gpu = ctx.mlp_infer(torch.from_numpy(lam).cuda()).cpu().numpy()
    w_ref, _ = M.forward(p, M.features(lam), bf16=True)
    err = np.max(np.abs(w_gpu - w_ref))
    _say(f"   max |w_gpu - w_oracle| = {err:.2e}")
    assert err <= 2e-5


def test_gradients_and_loss_match_oracle(lcf, ctx):
    _say("[mlp gradient parity]")
    ctx.mlp_init(11)
    p0 = ctx.mlp_get_params()
    p = M.unflatten(p0)
    lam, t = _spectra(200, 2)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ctx.mlp_train_step(torch.from_numpy(lam).cuda(), torch.from_numpy(t).cuda(), 0.0, loss_out=loss)
    torch.cuda.synchronize()
    g_gpu = M.unflatten(ctx.mlp_get_grads())
    z = M.features(lam)
    w, cache = M.forward(p, z, bf16=True)
    t64 = t.astype(np.float64)
    c = M.loss_weights(lam, t64)
    g_ref = M.backward(cache, t64, c)
    l_ref = M.loss(w, t64, c)
    _say(f"   loss gpu={loss.item():.6e} oracle={l_ref:.6e}")
    assert abs(loss.item() - l_ref) <= 1e-3 * abs(l_ref)
    for k in M.SHAPES:
        e = np.linalg.norm(g_gpu[k] - g_ref[k]) / max(np.linalg.norm(g_ref[k]), 1e-30)
        _say(f"   grad {k}: rel err {e:.2e}")
        assert e <= 1e-2, k
    # lr = 0 leaves the master weights unchanged
    assert np.array_equal(ctx.mlp_get_params(), p0)


def test_adam_step_matches_oracle(lcf, ctx):
    _say("[mlp adam step]")
    ctx.mlp_init(5)
    p = M.unflatten(ctx.mlp_get_params())
    lam, t = _spectra(128, 3)
    ctx.mlp_train_step(torch.from_numpy(lam).cuda(), torch.from_numpy(t).cuda(), 1e-3)
    torch.cuda.synchronize()
    got = M.unflatten(ctx.mlp_get_params())
    g = M.unflatten(ctx.mlp_get_grads())
    m = {k: np.zeros(s) for k, s in M.SHAPES.items()}
    v = {k: np.zeros(s) for k, s in M.SHAPES.items()}
    ref = {k: x.copy() for k, x in p.items()}
    M.adam_step(ref, {k: g[k].astype(np.float64) for k in g}, m, v, 1, 1e-3)
    for k in M.SHAPES:
        assert np.max(np.abs(got[k] - ref[k])) <= 1e-6, k


def test_checkpoint_roundtrip_and_crc(lcf, ctx):
    _say("[mlp checkpoint]")
    ctx.mlp_init(9)
    p = ctx.mlp_get_params()
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "w.ckpt")
        ctx.mlp_save(path)
        ctx.mlp_init(10)
        ctx.mlp_load(path)
        assert np.array_equal(ctx.mlp_get_params(), p)
        raw = bytearray(open(path, "rb").read())
        raw[100] ^= 0x55
        open(path, "wb").write(bytes(raw))
        ctx.mlp_init(10)
        with pytest.raises(lcf.LcfError) as ei:
            ctx.mlp_load(path)
        assert ei.value.status == 7
        assert not np.array_equal(ctx.mlp_get_params(), p)     # untouched by the failed load


def test_training_reduces_loss(lcf, ctx):
    _say("[mlp training]")
    ctx.mlp_init(3)
    lam, t = _spectra(2048, 4)
    lam_t, t_t = torch.from_numpy(lam).cuda(), torch.from_numpy(t).cuda()
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    losses = []
    for step in range(300):
        sl = slice((step % 4) * 512, (step % 4 + 1) * 512)
        ctx.mlp_train_step(lam_t[sl].contiguous(), t_t[sl].contiguous(), 2e-3, loss_out=loss)
        if step % 50 == 0 or step == 299:
            torch.cuda.synchronize()
            losses.append(loss.item())
    _say(f"   losses {['%.3e' % x for x in losses]}")
    assert losses[-1] < 0.2 * losses[0]


def test_filter_with_mlp_weights(lcf, ctx):
    _say("[filter with MLP weights]")
    ctx.mlp_init(21)
    p = M.unflatten(ctx.mlp_get_params())
    spec = synth.spec_clinical(1)
    iq, mask = synth.make_packet(spec)
    thr = lcf.Threshold(cut=lcf.CUT_MLP, shape=lcf.SHAPE_SIGMOID)
    ctx.set_option(lcf.OPT_MLP_GATE, -1)          # an untrained network: no gate
    try:
        io, pd, dg = ctx.filter(torch.from_numpy(iq).cuda(), 8, 8, thr, diag=True)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(lcf.OPT_MLP_GATE, 100)
    assert ctx.sync() == 0
    d = {k: v.cpu().numpy() for k, v in dg.items()}
    assert np.all((d["flags"] & lcf.FLAG_MLP_FALLBACK) == 0)
    w_ref, _ = M.forward(p, M.features(d["eigvals"]), bf16=True)
    assert np.max(np.abs(d["weights"] - w_ref)) <= 2e-5
    # the rest of the path with these weights, against the oracle forced to them
    res = O.filter_packet(iq, 8, 8, O.Threshold(cut=O.CUT_EXPLICIT, explicit_w=d["weights"].astype(np.float64)))
    e_fro = rel_fro(io.cpu().numpy(), res["iq_out"])
    emax, _, _, _ = pd_db_error(pd.cpu().numpy(), res["pd"], mask)
    _say(f"   rel_fro={e_fro:.2e} pd_db={emax:.2e}")
    assert e_fro <= 1e-5 and emax <= 0.1


@pytest.mark.parametrize("prec", [0, 1])
def test_mlp_gate_forced_and_consistent(lcf, ctx, prec):
    """Gate at 0 dB: every subset keeps the plain rule (flagged), and the
    outputs are bitwise those of the curvature rule with sigmoid weights. Gate
    at 0.1 dB: each subset's decision follows its exported prediction, and the
    prediction matches the oracle's on the GPU's eigenvalues and network
    weights (FP64 forward on the same BF16 weights)."""
    _say(f"[mlp gate prec={prec}]")
    ctx.mlp_init(21)
    p = M.unflatten(ctx.mlp_get_params())
    iq, mask = synth.make_packet(synth.spec_clinical(2))
    dev = torch.from_numpy(iq).cuda()
    thr = lcf.Threshold(cut=lcf.CUT_MLP, shape=lcf.SHAPE_SIGMOID)
    ctx.set_option(lcf.OPT_MLP_GATE, 0)
    try:
        io, pd, dg = ctx.filter(dev, 8, 8, thr, precision=prec, diag=True)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(lcf.OPT_MLP_GATE, 100)
    assert np.all(dg["flags"].cpu().numpy() & lcf.FLAG_MLP_FALLBACK)
    io_r, pd_r, dg_r = ctx.filter(dev, 8, 8, lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID),
                                  precision=prec, diag=True)
    torch.cuda.synchronize()
    assert torch.equal(io, io_r) and torch.equal(pd, pd_r)
    w_rule_gpu = dg_r["weights"].cpu().numpy()
    # default gate: decisions and predictions
    io, pd, dg = ctx.filter(dev, 8, 8, thr, precision=prec, diag=True)
    torch.cuda.synchronize()
    assert ctx.sync() == 0
    d = {k: v.cpu().numpy() for k, v in dg.items()}
    fb = (d["flags"] & lcf.FLAG_MLP_FALLBACK) != 0
    assert np.array_equal(fb, ~(d["mlp_gate"] < 0.1))
    w_net, _ = M.forward(p, M.features(d["eigvals"]), bf16=True)
    rule = O.Threshold(cut=O.CUT_KNEE, shape=O.SHAPE_SIGMOID)
    worst = 0.0
    for s in range(64):
        w_rule, _, _, _ = O.rule_weights(d["eigvals"][s], rule)
        g = O.mlp_gate(d["eigvals"][s], w_net[s], w_rule)
        if np.isinf(g) or np.isinf(d["mlp_gate"][s]):
            assert np.isinf(g) and np.isinf(d["mlp_gate"][s]), s
            continue
        worst = max(worst, abs(g - d["mlp_gate"][s]))
        if abs(g - 0.1) > 0.01:
            assert fb[s] == (g >= 0.1), s
        if fb[s]:
            assert np.array_equal(d["weights"][s], w_rule_gpu[s]), s
        else:
            assert np.allclose(d["weights"][s], w_net[s], atol=2e-5), s
    _say(f"   fallback {fb.mean():.2f}; prediction max |gpu - oracle| {worst:.2e} dB")
    assert worst <= 0.01


def test_mlp_fallback_for_other_nt(lcf, ctx):
    _say("[mlp fallback nt=64]")
    ctx.mlp_init(1)
    iq, _ = synth.make_packet(synth.PacketSpec(48, 40, 64, 50.0, 0.4, ((20, 3, 0.5),), seed=8))
    thr = lcf.Threshold(cut=lcf.CUT_MLP, shape=lcf.SHAPE_SIGMOID)
    _, _, dg = ctx.filter(torch.from_numpy(iq).cuda(), 2, 2, thr, diag=True)
    torch.cuda.synchronize()
    flags = dg["flags"].cpu().numpy()
    assert np.all(flags & lcf.FLAG_MLP_FALLBACK)
    lam = dg["eigvals"].cpu().numpy()
    for s in range(4):
        w_rule, _, _, _ = O.rule_weights(lam[s], O.Threshold(cut=O.CUT_KNEE, shape=O.SHAPE_SIGMOID))
        assert np.allclose(dg["weights"].cpu().numpy()[s], w_rule, atol=1e-6)


def test_learned_weights_gain_over_fixed_rule(lcf, ctx):
    """Train the network on the GPU (library kernels) to reproduce the per-packet
    CNR-searched beta of the curvature rule, then compare held-out packets: the
    network needs no search, and should beat the rule at the default beta."""
    _say("[mlp gain test]")
    from paper_2405_11105_amd import train_mlp as T
    lam, tgt, info = T.generate(ctx, lcf, "clinical", range(100, 148), (8, 8), lcf.PREC_FP32, workers=8)
    _say(f"   {lam.shape[0]} teacher spectra; best beta counts "
         f"{dict(zip(*np.unique([i['best_beta'] for i in info], return_counts=True)))}")
    ctx.mlp_init(2)
    hist = T.train(ctx, lam, tgt, epochs=60, batch=512, lr=3e-3)
    _say(f"   loss first/last epoch {hist[0]:.3e} / {hist[-1]:.3e}")
    rows = T.evaluate(ctx, lcf, "clinical", range(200, 212), (8, 8), lcf.PREC_FP32, workers=8)
    rule = np.array([r["cnr_rule"] for r in rows])
    mlp_ = np.array([r["cnr_mlp"] for r in rows])
    teach = np.array([r["cnr_teacher"] for r in rows])
    _say(f"   held-out CNR dB: rule(beta=1) {rule.mean():.2f}  mlp {mlp_.mean():.2f}  searched-beta {teach.mean():.2f}")
    _say(f"   per packet gain mlp-rule: {np.round(mlp_ - rule, 2).tolist()}")
    _say(f"   behind the 0.1 dB gate: CNR {np.mean([r['cnr_gated'] for r in rows]):.2f} dB, fallback "
         f"{np.mean([r['fallback_rate'] for r in rows]):.2f}, PD vs rule p99 "
         f"{np.mean([r['pd_db_gated_vs_rule_p99'] for r in rows]):.3f} dB")
    assert hist[-1] < hist[0]
    assert mlp_.mean() > rule.mean()
