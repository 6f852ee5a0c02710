"""Parity of the benchmark's own configuration against the FP64 oracle: four
512 x 256 x 128 packets, 16 x 16 Gaussian windows (256 subsets each), learned
weights from the committed network behind the default 0.1 dB gate (the plain
curvature rule with sigmoid weights as fallback), all packets in one batched
call replayed from a captured hipGraph, in split-BF16 and in FP32. The packets
are held out from the network's training seeds."""
import os

import numpy as np
import pytest

import oracle as O
from oracle import mlp as M
import synth
from parity import say, rel_fro, pd_db_error, knee_tie

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CKPT = os.path.join(ROOT, "paper_2405_11105_amd", "weights", "mlp_512x256x128.ckpt")
SEEDS = [20000, 20001, 20002, 20003]       # the benchmark's packets
GRID = (16, 16)
GATE_DB = 0.1
RULE = O.Threshold(cut=O.CUT_KNEE, shape=O.SHAPE_SIGMOID)


@pytest.fixture(scope="module")
def packets():
    return [synth.make_packet(synth.spec_learned(s)) for s in SEEDS]


@pytest.fixture(scope="module")
def network(lcf):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    c = lcf.Context(0)
    c.mlp_load(CKPT)
    params = M.unflatten(c.mlp_get_params())
    c.close()
    return params


@pytest.fixture(scope="module")
def oracle_out(packets, network):
    thr = O.Threshold(cut=O.CUT_MLP, shape=O.SHAPE_SIGMOID, mlp_gate_db=GATE_DB,
                      mlp=lambda lam: M.forward(network, M.features(lam), bf16=True)[0][0])
    out = []
    for i, (iq, _) in enumerate(packets):
        say(f"   oracle packet {i}")
        out.append(O.filter_packet(iq, GRID[0], GRID[1], thr))
    return out


@pytest.mark.parametrize("prec", [1, 0])
def test_benchmark_configuration_vs_oracle(lcf, packets, network, oracle_out, prec):
    tol = 1e-5 if prec == lcf.PREC_FP32 else 1e-3
    say(f"[benchmark configuration prec={prec}]")
    thr = lcf.Threshold(cut=lcf.CUT_MLP, shape=lcf.SHAPE_SIGMOID)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        dev = [torch.from_numpy(iq).cuda() for iq, _ in packets]
        gctx = lcf.Context(0, use_graph=1)
        ectx = lcf.Context(0)
        try:
            gctx.mlp_load(CKPT)
            ectx.mlp_load(CKPT)
            outs = [(torch.empty_like(d), torch.empty(d.shape[1:], dtype=torch.float32, device="cuda"))
                    for d in dev]
            first = None
            for rep in range(3):
                gctx.filter_batch(dev, [GRID] * 4, thr, precision=prec, outs=outs)
                st.synchronize()
                got = [(io.cpu().numpy(), pd.cpu().numpy()) for io, pd in outs]
                if first is None:
                    first = got
                else:
                    for a, b in zip(first, got):
                        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), rep
                _ = (dev[0].abs() ** 2).sum().item()          # eager work between replays
            assert gctx.sync() == 0
            for i, (iq, mask) in enumerate(packets):
                io1, pd1, dg = ectx.filter(dev[i], GRID[0], GRID[1], thr, precision=prec, diag=True)
                st.synchronize()
                assert ectx.sync() == 0
                assert np.array_equal(io1.cpu().numpy(), first[i][0]) and np.array_equal(pd1.cpu().numpy(), first[i][1])
                d = {k: v.cpu().numpy() for k, v in dg.items()}
                res = oracle_out[i]
                fb = (d["flags"] & lcf.FLAG_MLP_FALLBACK) != 0
                assert np.array_equal(fb, ~(d["mlp_gate"] < GATE_DB))
                # the network's weights on the GPU's eigenvalues, in FP64 on the same BF16 weights
                w_ref, _ = M.forward(network, M.features(d["eigvals"]), bf16=True)
                ew, gerr, forced = 0.0, 0.0, False
                for s in range(GRID[0] * GRID[1]):
                    lam = d["eigvals"][s]
                    w_rule, k_rule, curv, _ = O.rule_weights(lam, RULE)
                    g = O.mlp_gate(lam, w_ref[s], w_rule)
                    assert np.isinf(g) == np.isinf(d["mlp_gate"][s]), s
                    if np.isfinite(g):
                        gerr = max(gerr, abs(g - d["mlp_gate"][s]))
                    if abs(g - GATE_DB) > 0.01:
                        assert fb[s] == (g >= GATE_DB), s
                    if fb[s]:
                        if d["k"][s] != k_rule:
                            assert knee_tie(curv, int(d["k"][s]), k_rule), s
                        else:
                            assert np.allclose(d["weights"][s], w_rule, atol=1e-6), s
                    else:
                        ew = max(ew, float(np.max(np.abs(d["weights"][s] - w_ref[s]))))
                    # the oracle's own decision (on its eigenvalues) may differ only at a tie
                    fo = (res["flags"][s] & O.FLAG_MLP_FALLBACK) != 0
                    if fo != fb[s] or (fb[s] and d["k"][s] != res["k"][s]):
                        forced = True
                say(f"   packet {i}: fallback {fb.mean():.3f}, gate prediction |gpu - oracle| {gerr:.1e} dB, "
                    f"forced={forced}")
                assert gerr <= 0.01
                if forced:
                    res = O.filter_packet(iq, GRID[0], GRID[1],
                                          O.Threshold(cut=O.CUT_EXPLICIT, explicit_w=d["weights"].astype(np.float64)))
                lam_err = float(np.max(np.abs(d["eigvals"] - np.array(res["lam"])) / np.array(res["lam"])[:, :1]))
                e_fro = rel_fro(first[i][0], res["iq_out"])
                emax, e99, e999, npx = pd_db_error(first[i][1], res["pd"], mask)
                say(f"   packet {i}: rel_fro={e_fro:.3e} pd_db max={emax:.2e} p99={e99:.2e} n={npx} "
                    f"weights {ew:.1e} eigenvalues {lam_err:.1e} (of lambda_1)")
                assert ew <= 2e-5
                assert e_fro <= tol and emax <= 0.1
        finally:
            gctx.close()
            ectx.close()
