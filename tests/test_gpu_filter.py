"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle."""
import sys

import numpy as np
import pytest

import oracle as O
import synth
from parity import rel_fro, run_gpu as _run, oracle_thr as _oracle_thr, \
    check_end_to_end as _check_end_to_end

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


# ------------------------------------------------------------------ EVD

@pytest.mark.parametrize("nt", [32, 64, 100, 128, 200])
def test_heevd_circulant_closed_form(lcf, ctx, nt):
    _say(f"[heevd circulant nt={nt}]")
    rng = np.random.default_rng(nt)
    lam = 10.0 ** rng.uniform(-8.0, 0.0, size=(3, nt))
    mats = []
    for b in range(3):
        col = np.fft.ifft(lam[b])
        idx = (np.arange(nt)[:, None] - np.arange(nt)[None, :]) % nt
        mats.append(col[idx])
    a = np.ascontiguousarray(np.stack(mats))
    # log-uniform spectra over 8 decades with equal column norms are a slow case
    # for one-sided Jacobi: allow more sweeps than the filter's default cap
    ctx.set_option(lcf.OPT_MAX_SWEEPS, 100)
    try:
        w, v, sw = ctx.heevd(torch.from_numpy(a).cuda())
        torch.cuda.synchronize()
    finally:
        ctx.set_option(lcf.OPT_MAX_SWEEPS, 30)
    w, v, sw = w.cpu().numpy(), v.cpu().numpy(), sw.cpu().numpy()
    _say(f"   sweeps {sw.tolist()}")
    for b in range(3):
        ref = np.sort(lam[b])[::-1]
        assert np.max(np.abs(w[b] - ref)) <= 1e-13, (b, np.max(np.abs(w[b] - ref)))
        assert np.linalg.norm(v[b].conj().T @ v[b] - np.eye(nt)) <= 1e-10
        res = np.linalg.norm(a[b] @ v[b] - v[b] * w[b][None, :])
        # backward-stable bound: a small multiple of nt * u * ||R||
        assert res <= 10 * nt * 1.1102230246251565e-16 * np.linalg.norm(a[b]), res
    assert np.all(sw > 0) and np.all(sw < 100)


def test_heevd_random_psd_vs_eigh(lcf, ctx):
    _say("[heevd random psd]")
    rng = np.random.default_rng(5)
    nt = 48
    x = rng.standard_normal((4, 200, nt)) + 1j * rng.standard_normal((4, 200, nt))
    a = np.ascontiguousarray(np.einsum("bki,bkj->bij", x.conj(), x))
    w, v, _ = ctx.heevd(torch.from_numpy(a).cuda())
    w = w.cpu().numpy()
    for b in range(4):
        ref = np.linalg.eigvalsh(a[b])[::-1]
        assert np.allclose(w[b], ref, rtol=1e-12, atol=1e-12 * ref[0])


# ------------------------------------------------------------------ covariance

def test_covariance_integer_exact(lcf, ctx):
    _say("[cov integer exact]")
    rng = np.random.default_rng(3)
    nt, ny, nx = 32, 24, 20
    iq = (rng.integers(-8, 9, size=(nt, ny, nx)) + 1j * rng.integers(-8, 9, size=(nt, ny, nx))).astype(np.complex64)
    thr = lcf.Threshold(cut=lcf.CUT_FIXED_K, k_fixed=2, deflate_rho=0.0)
    iq_t = torch.from_numpy(iq).cuda()
    _, _, dg = ctx.filter(iq_t, 1, 1, thr, sigma_frac=0.0, diag_cov=True)
    cov = dg["cov"].cpu().numpy()[0]
    c = O.casorati(iq)
    ref = O.covariance(c)
    assert np.array_equal(cov, ref)


def test_covariance_windowed_matches_oracle(lcf, ctx):
    _say("[cov windowed 64x64x32 3x3]")
    iq, _ = synth.make_packet(synth.spec_small(0))
    thr = lcf.Threshold(cut=lcf.CUT_FIXED_K, k_fixed=4)
    iq_t = torch.from_numpy(iq).cuda()
    _, _, dg = ctx.filter(iq_t, 3, 3, thr, diag_cov=True)
    cov = dg["cov"].cpu().numpy()
    res = O.filter_packet(iq, 3, 3, _oracle_thr(thr))
    for d in range(9):
        e = np.linalg.norm(cov[d] - res["cov"][d]) / np.linalg.norm(res["cov"][d])
        assert e <= 1e-6, (d, e)


# ------------------------------------------------------------------ end to end

def test_small_fixed_k(lcf, ctx):
    iq, mask = synth.make_packet(synth.spec_small(0))
    thr = lcf.Threshold(cut=lcf.CUT_FIXED_K, k_fixed=4)
    _check_end_to_end(lcf, ctx, iq, mask, 3, 3, thr, 1e-5, 0.1, "small fixed-k")


@pytest.mark.parametrize("shape", [0, 1])
def test_clinical_knee(lcf, ctx, shape):
    spec = synth.spec_clinical(0)
    iq, mask = synth.make_packet(spec)
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=shape)
    _check_end_to_end(lcf, ctx, iq, mask, 8, 8, thr, 1e-5, 0.1, f"clinical knee shape={shape}")


def test_ragged_nt100_small_grid(lcf, ctx):
    spec = synth.PacketSpec(72, 50, 100, 50.0, 0.5, ((20, 3, 0.4), (51, 2, 0.8)), seed=77)
    iq, mask = synth.make_packet(spec)
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
    _check_end_to_end(lcf, ctx, iq, mask, 3, 2, thr, 1e-5, 0.1, "ragged nt=100")


@pytest.mark.parametrize("nt", [80, 150])
@pytest.mark.parametrize("prec", [0, 1])
def test_ragged_frame_counts_80_150(lcf, ctx, nt, prec):
    # 80 frames fall in the 96 class (16 padding frames), 150 in the 160 class;
    # both are ragged in the pixels as well
    spec = synth.PacketSpec(90, 70, nt, 50.0, 0.4, ((25, 3, 0.3), (60, 4, 0.7)), seed=500 + nt)
    iq, mask = synth.make_packet(spec)
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
    tol = 1e-5 if prec == lcf.PREC_FP32 else 1e-3
    _check_end_to_end(lcf, ctx, iq, mask, 3, 2, thr, tol, 0.1, f"nt={nt} prec={prec}", precision=prec)


@pytest.mark.parametrize("nt", [4, 208])
@pytest.mark.parametrize("prec", [0, 1])
def test_frame_count_limits(lcf, ctx, nt, prec):
    # the shortest packet the library accepts (28 padding frames in the 32 class,
    # tissue rank capped by nt) and the longest (the 208 class exactly filled)
    spec = synth.PacketSpec(48, 40, nt, 50.0, 0.4, ((20, 3, 0.5),), seed=900 + nt)
    iq, mask = synth.make_packet(spec)
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
    tol = 1e-5 if prec == lcf.PREC_FP32 else 1e-3
    _check_end_to_end(lcf, ctx, iq, mask, 2, 2, thr, tol, 0.1, f"nt={nt} prec={prec}", precision=prec)


def test_batch_argument_errors(lcf, ctx):
    _say("[batch argument errors]")
    thr = lcf.Threshold(cut=lcf.CUT_KNEE)
    with pytest.raises(lcf.LcfError) as ei:
        ctx.filter_batch([], [], thr)
    assert ei.value.status == 1     # LCF_ERR_INVALID_ARG
    # caller-given weights without a weight array
    iq = torch.from_numpy(synth.make_packet(synth.spec_small(3))[0]).cuda()
    with pytest.raises(lcf.LcfError) as ei:
        ctx.filter_batch([iq], [(2, 2)], lcf.Threshold(cut=lcf.CUT_EXPLICIT))
    assert ei.value.status == 1     # LCF_ERR_INVALID_ARG


@pytest.mark.parametrize("prec", [0, 1])
def test_clinical_median_rule(lcf, ctx, prec):
    # method 3 (Eq. 7) at the clinical shape with beta = 30, which puts the cut
    # at the tissue / blood transition of these packets (k = 3 to 7; the
    # curvature rule gives 5 to 19); the paper's own beta follows.
    iq, mask = synth.make_packet(synth.spec_clinical(1))
    thr = lcf.Threshold(cut=lcf.CUT_MEDIAN, beta_median=30.0)
    tol = 1e-5 if prec == lcf.PREC_FP32 else 1e-3
    _check_end_to_end(lcf, ctx, iq, mask, 8, 8, thr, tol, 0.1, f"clinical median prec={prec}", precision=prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_clinical_median_rule_paper_beta(lcf, ctx, prec):
    # method 3 (Eq. 7) at the scaling factor of the paper's Fig. 2a example, fitted
    # to the paper's data: here it cuts 35 to 52 components deep, inside the noise
    # floor, where the eigen-gap at the cut is about 3e-10 lambda_1, so the
    # filtered IQ follows the rounding of the bulk Gram C'^H C' over that gap
    # (the FP32 pass-2 Gram sums its MFMA batches in FP64 for this)
    iq, mask = synth.make_packet(synth.spec_clinical(1))
    thr = lcf.Threshold(cut=lcf.CUT_MEDIAN, beta_median=1.43)
    tol = 1e-5 if prec == lcf.PREC_FP32 else 1e-3
    _check_end_to_end(lcf, ctx, iq, mask, 8, 8, thr, tol, 0.1, f"clinical median beta=1.43 prec={prec}",
                      precision=prec)


def test_median_rule_odd_frame_count_sigmoid(lcf, ctx):
    # an odd count takes the middle eigenvalue itself; soft weights centred on k
    spec = synth.PacketSpec(80, 64, 45, 50.0, 0.5, ((30, 3, 0.6),), seed=45)
    iq, mask = synth.make_packet(spec)
    thr = lcf.Threshold(cut=lcf.CUT_MEDIAN, beta_median=30.0, shape=lcf.SHAPE_SIGMOID)
    _check_end_to_end(lcf, ctx, iq, mask, 3, 3, thr, 1e-5, 0.1, "median odd nt=45 sigmoid")


@pytest.mark.parametrize("prec", [0, 1])
def test_clinical_slope_rule(lcf, ctx, prec):
    # the slope rule at the clinical shape with the threshold of the paper's
    # Fig. 2c example (the turning point falls after the tissue components)
    iq, mask = synth.make_packet(synth.spec_clinical(2))
    thr = lcf.Threshold(cut=lcf.CUT_SLOPE, slope_thr=1.1)
    tol = 1e-5 if prec == lcf.PREC_FP32 else 1e-3
    _check_end_to_end(lcf, ctx, iq, mask, 8, 8, thr, tol, 0.1, f"clinical slope prec={prec}", precision=prec)


def test_slope_rule_odd_frame_count_sigmoid(lcf, ctx):
    spec = synth.PacketSpec(80, 64, 45, 50.0, 0.5, ((30, 3, 0.6),), seed=46)
    iq, mask = synth.make_packet(spec)
    thr = lcf.Threshold(cut=lcf.CUT_SLOPE, slope_thr=0.3, shape=lcf.SHAPE_SIGMOID)
    _check_end_to_end(lcf, ctx, iq, mask, 3, 3, thr, 1e-5, 0.1, "slope nt=45 sigmoid")


@pytest.mark.parametrize("prec", [0, 1])
def test_clinical_power_weights(lcf, ctx, prec):
    # method 6 (Eq. 10) with the order of the paper's Fig. 2g example
    iq, mask = synth.make_packet(synth.spec_clinical(3))
    thr = lcf.Threshold(cut=lcf.CUT_POWER, beta_power=2.0)
    tol = 1e-5 if prec == lcf.PREC_FP32 else 1e-3
    _check_end_to_end(lcf, ctx, iq, mask, 8, 8, thr, tol, 0.1, f"clinical power prec={prec}", precision=prec)


def test_power_weights_odd_frame_count(lcf, ctx):
    spec = synth.PacketSpec(80, 64, 45, 50.0, 0.5, ((30, 3, 0.6),), seed=47)
    iq, mask = synth.make_packet(spec)
    thr = lcf.Threshold(cut=lcf.CUT_POWER, beta_power=1.0)
    _check_end_to_end(lcf, ctx, iq, mask, 3, 3, thr, 1e-5, 0.1, "power nt=45")


def test_all_ones_weights_return_input(lcf, ctx):
    _say("[all-ones identity]")
    iq, _ = synth.make_packet(synth.spec_small(1))
    thr = lcf.Threshold(cut=lcf.CUT_EXPLICIT)
    ew = torch.ones((9, 32), dtype=torch.float32)
    io, _, _ = ctx.filter(torch.from_numpy(iq).cuda(), 3, 3, thr, explicit_w=ew)
    io = io.cpu().numpy()
    assert rel_fro(io, iq) <= 1e-6


def test_global_window_is_svd_filter(lcf, ctx):
    _say("[global flat window]")
    iq, mask = synth.make_packet(synth.spec_small(2))
    thr = lcf.Threshold(cut=lcf.CUT_FIXED_K, k_fixed=3)
    io, pd, _ = _run(lcf, ctx, iq, 1, 1, thr, sigma_frac=0.0)
    c = O.casorati(iq)
    u, s, vh = np.linalg.svd(c, full_matrices=False)
    chat = c - (u[:, :3] * s[:3]) @ vh[:3]
    assert rel_fro(O.casorati(io), chat) <= 1e-5


def test_sequential_schedule_matches_batched(lcf, ctx):
    _say("[sequential vs batched]")
    iq, _ = synth.make_packet(synth.spec_small(4))
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
    iq_t = torch.from_numpy(iq).cuda()
    a_io, a_pd, _ = ctx.filter(iq_t, 3, 3, thr)
    ctx.set_option(lcf.OPT_SCHEDULE, 1)
    try:
        b_io, b_pd, _ = ctx.filter(iq_t, 3, 3, thr)
    finally:
        ctx.set_option(lcf.OPT_SCHEDULE, 0)
    torch.cuda.synchronize()
    assert torch.equal(a_io, b_io) and torch.equal(a_pd, b_pd)


def test_deterministic_reruns(lcf, ctx):
    _say("[determinism]")
    iq, _ = synth.make_packet(synth.spec_small(5))
    thr = lcf.Threshold(cut=lcf.CUT_KNEE)
    iq_t = torch.from_numpy(iq).cuda()
    a = ctx.filter(iq_t, 3, 3, thr)
    b = ctx.filter(iq_t, 3, 3, thr)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_batch_mixed_shapes_matches_single(lcf, ctx):
    _say("[batch mixed shapes]")
    specs = [synth.PacketSpec(64, 48, 32, 50.0, 0.3, ((20, 3, 0.5),), seed=11),
             synth.PacketSpec(40, 56, 64, 50.0, 0.3, ((15, 2, 0.2),), seed=12),
             synth.PacketSpec(64, 48, 32, 45.0, 0.6, ((30, 4, 0.9),), seed=13),
             synth.PacketSpec(56, 40, 80, 50.0, 0.4, ((25, 3, 0.5),), seed=14)]
    grids = [(2, 2), (3, 2), (2, 3), (3, 3)]
    iqs = [torch.from_numpy(synth.make_packet(s)[0]).cuda() for s in specs]
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
    ios, pds = ctx.filter_batch(iqs, grids, thr, iq_out=True)
    for i, (iq, g) in enumerate(zip(iqs, grids)):
        io1, pd1, _ = ctx.filter(iq, g[0], g[1], thr)
        torch.cuda.synchronize()
        assert torch.equal(ios[i], io1) and torch.equal(pds[i], pd1), i


def test_nonfinite_input_reported(lcf, ctx):
    _say("[nonfinite input]")
    iq, _ = synth.make_packet(synth.spec_small(6))
    iq[3, 10, 10] = np.nan
    thr = lcf.Threshold(cut=lcf.CUT_FIXED_K, k_fixed=2)
    ctx.filter(torch.from_numpy(iq).cuda(), 2, 2, thr)
    assert ctx.sync() == 5
    assert ctx.sync() == 0


# ------------------------------------------------------------------ split-BF16 path

def test_covariance_integer_exact_bf16x3(lcf, ctx):
    _say("[cov integer exact bf16x3]")
    rng = np.random.default_rng(4)
    nt, ny, nx = 32, 24, 20
    iq = (rng.integers(-8, 9, size=(nt, ny, nx)) + 1j * rng.integers(-8, 9, size=(nt, ny, nx))).astype(np.complex64)
    thr = lcf.Threshold(cut=lcf.CUT_FIXED_K, k_fixed=2, deflate_rho=0.0)
    _, _, dg = ctx.filter(torch.from_numpy(iq).cuda(), 1, 1, thr, precision=lcf.PREC_BF16X3, sigma_frac=0.0,
                          diag_cov=True)
    cov = dg["cov"].cpu().numpy()[0]
    assert np.array_equal(cov, O.covariance(O.casorati(iq)))


def test_small_fixed_k_bf16x3(lcf, ctx):
    iq, mask = synth.make_packet(synth.spec_small(0))
    thr = lcf.Threshold(cut=lcf.CUT_FIXED_K, k_fixed=4)
    _check_end_to_end(lcf, ctx, iq, mask, 3, 3, thr, 1e-3, 0.1, "small fixed-k bf16x3", precision=lcf.PREC_BF16X3)


@pytest.mark.parametrize("shape", [0, 1])
def test_precision_60db_bf16x3(lcf, ctx, shape):
    spec = synth.spec_precision(0)
    iq, mask = synth.make_packet(spec)
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=shape)
    _check_end_to_end(lcf, ctx, iq, mask, 8, 8, thr, 1e-3, 0.1, f"60 dB bf16x3 shape={shape}",
                      precision=lcf.PREC_BF16X3)


def test_precision_60db_fp32(lcf, ctx):
    spec = synth.spec_precision(1)
    iq, mask = synth.make_packet(spec)
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
    _check_end_to_end(lcf, ctx, iq, mask, 8, 8, thr, 1e-5, 0.1, "60 dB fp32")


def test_graph_replay_matches_eager(lcf, ctx):
    _say("[hipGraph replay]")
    iqs = [torch.from_numpy(synth.make_packet(synth.spec_small(s))[0]).cuda() for s in (7, 8)]
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ref = [ctx.filter(iq, 3, 3, thr) for iq in iqs]
        st.synchronize()
        gctx = lcf.Context(0, use_graph=1)
        try:
            for rep in range(4):
                for i, iq in enumerate(iqs):
                    io, pd, _ = gctx.filter(iq, 3, 3, thr)
                    st.synchronize()
                    assert torch.equal(io, ref[i][0]) and torch.equal(pd, ref[i][1]), (rep, i)
                # eager work of the program between replays
                _ = (iqs[0].abs() ** 2).sum().item()
                ctx.filter(iqs[1], 2, 2, thr)
                st.synchronize()
            assert gctx.sync() == 0
        finally:
            gctx.close()


def test_graph_cache_keys_on_median_beta(lcf, ctx):
    # the rule parameters are baked into a captured graph: a call that changes
    # only beta of Eq. 7 must not replay the graph of another beta
    _say("[hipGraph median beta]")
    iq = torch.from_numpy(synth.make_packet(synth.spec_small(9))[0]).cuda()
    thrs = [lcf.Threshold(cut=lcf.CUT_MEDIAN, beta_median=b) for b in (1.43, 20.0)]
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ref = [ctx.filter(iq, 3, 3, t, diag=True) for t in thrs]
        st.synchronize()
        assert not np.array_equal(ref[0][2]["k"].cpu().numpy(), ref[1][2]["k"].cpu().numpy())
        gctx = lcf.Context(0, use_graph=1)
        try:
            for rep in range(3):
                for i, t in enumerate(thrs):
                    io, pd, _ = gctx.filter(iq, 3, 3, t)
                    st.synchronize()
                    assert torch.equal(pd, ref[i][1]), (rep, i)
            assert gctx.sync() == 0
        finally:
            gctx.close()


@pytest.mark.parametrize("nt", [128, 80, 150, 200, 4, 33, 65, 66, 127])
def test_evd_tridiagonal_matches_jacobi(lcf, ctx, nt):
    """The two subset eigen-solvers give the same filter (FP32 path); 80 frames
    run the 6-wave shapes of both (96-frame class); 150 and 200 frames run the
    global-memory Householder reduction (160 and 208 classes) against the
    LDS / global Jacobi. The register reduction's edges: 4 frames (two
    reflectors, 2 waves), 33 (4 waves), 65 (the last step before the reduction
    drops its first row block), 66 (one step after it), 127 (the last steps
    leave some waves without columns to update)."""
    _say(f"[tridiagonal vs Jacobi EVD nt={nt}]")
    iq, mask = synth.make_packet(synth.spec_clinical(2, nt=nt))
    dev = torch.from_numpy(iq).cuda()
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
    io_t, pd_t, d_t = ctx.filter(dev, 8, 8, thr, diag=True)
    ctx.set_option(lcf.OPT_EVD, lcf.EVD_JACOBI)
    try:
        io_j, pd_j, d_j = ctx.filter(dev, 8, 8, thr, diag=True)
    finally:
        ctx.set_option(lcf.OPT_EVD, lcf.EVD_TRIDIAGONAL)
    torch.cuda.synchronize()
    assert ctx.sync() == 0
    lt, lj = d_t["eigvals"].cpu().numpy(), d_j["eigvals"].cpu().numpy()
    e_lam = float(np.max(np.abs(lt - lj) / lj[:, :1]))
    e_io = float(torch.linalg.vector_norm(io_t - io_j) / torch.linalg.vector_norm(io_j))
    e_pd = float(torch.max(torch.abs(pd_t - pd_j) / pd_j))
    fb = int(((d_t["flags"] & lcf.FLAG_EVD_JACOBI) != 0).sum())
    _say(f"   eigenvalues {e_lam:.1e} (of lambda_1), iq {e_io:.1e}, pd {e_pd:.1e}, Jacobi fallbacks {fb}")
    assert fb == 0                       # every subset took the tridiagonal path
    assert e_lam <= 1e-12 and e_io <= 1e-7 and e_pd <= 1e-6
    assert np.array_equal(d_t["k"].cpu().numpy(), d_j["k"].cpu().numpy())


@pytest.mark.parametrize("nt", [128, 127])
def test_evd_tridiagonal_batch_matches_jacobi(lcf, ctx, nt):
    """Four packets on 16 x 16 grids (1024 subsets in one batch, every
    work-group slot of the EVD kernels filled): the filtered packets of the
    tridiagonal solver against Jacobi's."""
    _say(f"[tridiagonal vs Jacobi EVD, 1024-subset batch, nt={nt}]")
    dev = [torch.from_numpy(synth.make_packet(synth.spec_clinical(p, nt=nt))[0]).cuda() for p in range(4)]
    grids = [(16, 16)] * 4
    thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
    io_t, _ = ctx.filter_batch(dev, grids, thr, iq_out=True)
    ctx.set_option(lcf.OPT_EVD, lcf.EVD_JACOBI)
    try:
        io_j, _ = ctx.filter_batch(dev, grids, thr, iq_out=True)
    finally:
        ctx.set_option(lcf.OPT_EVD, lcf.EVD_TRIDIAGONAL)
    torch.cuda.synchronize()
    assert ctx.sync() == 0
    for p in range(4):
        e = float(torch.linalg.vector_norm(io_t[p] - io_j[p]) / torch.linalg.vector_norm(io_j[p]))
        _say(f"   packet {p}: iq {e:.1e}")
        assert e <= 1e-7, p


@pytest.mark.parametrize("nt", [32, 150])
def test_evd_rank_deficient_falls_back_to_jacobi(lcf, ctx, nt):
    """Boxes of at most 30 pixels and 32 (150) frames: every subset covariance is
    singular with a repeated zero eigenvalue, and the slow sigmoid (beta 0.5 from
    k = 3) gives those components weights other than 1, so the projector needs
    their vectors: the tridiagonal solver (the register one, the global-memory
    one) hands the subset to Jacobi."""
    _say(f"[rank-deficient subsets nt={nt}]")
    spec = synth.PacketSpec(6, 5, nt, 30.0, 0.3, ((3, 1, 0.5),), seed=21)
    iq, mask = synth.make_packet(spec)
    thr = lcf.Threshold(cut=lcf.CUT_FIXED_K, shape=lcf.SHAPE_SIGMOID, k_fixed=3, beta_sigmoid=0.5)
    io, pd, d = _run(lcf, ctx, iq, 2, 2, thr)
    assert np.all(d["flags"] & lcf.FLAG_EVD_JACOBI)
    res = O.filter_packet(iq, 2, 2, _oracle_thr(thr))
    e = rel_fro(io, res["iq_out"])
    _say(f"   rel_fro={e:.2e}")
    assert e <= 1e-5


def test_evd_near_degenerate_noise_needs_no_fallback(lcf, ctx):
    """The same singular subsets with the hard cut at k = 3: the repeated zero
    eigenvalues get weight 1, their vectors never enter the projector, so no
    subset takes the Jacobi path and the output still matches the oracle."""
    _say("[rank-deficient subsets, hard cut]")
    spec = synth.PacketSpec(6, 5, 32, 30.0, 0.3, ((3, 1, 0.5),), seed=21)
    iq, mask = synth.make_packet(spec)
    thr = lcf.Threshold(cut=lcf.CUT_FIXED_K, k_fixed=3)
    io, pd, d = _run(lcf, ctx, iq, 2, 2, thr)
    assert not np.any(d["flags"] & lcf.FLAG_EVD_JACOBI)
    res = O.filter_packet(iq, 2, 2, _oracle_thr(thr))
    e = rel_fro(io, res["iq_out"])
    _say(f"   rel_fro={e:.2e}")
    assert e <= 1e-5
