"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
hand-worked values, closed forms, LAPACK/SVD identities and brute force."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from oracle.jacobi import jacobi_eigh
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_packet(nt, ny, nx, seed=0, integer=False):
    rng = np.random.default_rng(seed)
    if integer:
        re = rng.integers(-8, 9, size=(nt, ny, nx))
        im = rng.integers(-8, 9, size=(nt, ny, nx))
        return (re + 1j * im).astype(np.complex64)
    z = rng.standard_normal((nt, ny, nx)) + 1j * rng.standard_normal((nt, ny, nx))
    return z.astype(np.complex64)


def _low_rank_packet(nt, ny, nx, rank, seed=1, tissue_amp=300.0, blood=0.0, dtype=np.complex64):
    """Tissue of exact rank `rank`: sum_j a_j(x) f_j(t), plus optional blood noise."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((rank, ny * nx)) + 1j * rng.standard_normal((rank, ny * nx))
    f = rng.standard_normal((rank, nt)) + 1j * rng.standard_normal((rank, nt))
    c = tissue_amp * (a.T @ f)                       # [npix][nt]
    c += blood * (rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape))
    return np.ascontiguousarray(c.T.reshape(nt, ny, nx)).astype(dtype)


# ---------------------------------------------------------------- windows (Eq. 11)

def test_window_boxes_hand_values():
    # 64 px, 3 windows: spacing 64/3, centre of window 0 = 0.5*64/3 - 0.5 = 10.1666..,
    # sigma = 64/9 = 7.111..; +-6 sigma box = [10.1667-42.6667, 10.1667+42.6667] = [-32.5, 52.83]
    wins = O.window_boxes(64, 64, 3, 3, 1.0 / 3.0, 6.0)
    w0 = wins[0]
    assert abs(w0.cy - 10.166666666666666) < 1e-12 and abs(w0.sy - 7.111111111111111) < 1e-12
    assert (w0.y0, w0.y1, w0.x0, w0.x1) == (0, 52, 0, 52)
    w4 = wins[4]                       # centre window: centre 31.5, box [-11.17, 74.17] -> [0, 63]
    assert abs(w4.cy - 31.5) < 1e-12 and (w4.y0, w4.y1) == (0, 63)
    # index order d = a*gx + b: window 1 moves along x
    assert wins[1].cy == w0.cy and wins[1].cx > w0.cx
    # truncation at 1 sigma around 31.5 with sigma 7.111: [24.39, 38.61] -> [25, 38]
    w = O.window_boxes(64, 64, 3, 3, 1.0 / 3.0, 1.0)[4]
    assert (w.y0, w.y1) == (25, 38)


def test_window_table_values():
    win = O.window_boxes(64, 64, 3, 3, 1.0 / 3.0, 6.0)[4]
    t = O.window_table(win, 64, 64)
    # value at (31, 32): offsets -0.5, +0.5 -> exp(-(0.25+0.25)/(2*sigma^2))
    s = 64.0 / 9.0
    assert abs(t[31, 32] - math.exp(-0.5 / (2 * s * s))) < 1e-15
    assert np.allclose(t, t[::-1, ::-1])           # symmetric about the half-integer centre
    assert t.max() <= 1.0
    # flat global window
    flat = O.window_boxes(8, 6, 1, 1, 0.0, 6.0)[0]
    assert np.all(O.window_table(flat, 8, 6) == 1.0)


# ---------------------------------------------------------------- covariance (Eqs 1, 12)

def test_covariance_integer_bruteforce():
    iq = _rand_packet(6, 5, 4, seed=3, integer=True)
    c = O.casorati(iq)
    r = O.covariance(c)
    nt = iq.shape[0]
    for j in range(nt):
        for k in range(nt):
            acc = 0j
            for y in range(iq.shape[1]):
                for x in range(iq.shape[2]):
                    acc += complex(iq[j, y, x]).conjugate() * complex(iq[k, y, x])
            assert r[j, k] == acc                   # exact: small integers
    assert np.array_equal(r, r.conj().T)


def test_covariance_equals_squared_singular_values():
    # Eq. 3: eigenvalues of C_w^H C_w are the squared singular values of C_w
    iq = _rand_packet(10, 9, 7, seed=4)
    win = O.window_boxes(9, 7, 2, 2, 1.0 / 3.0, 6.0)[1]
    w = O.window_table(win, 9, 7).reshape(-1)
    cw = w[:, None] * O.casorati(iq)
    lam, _ = O.evd(O.covariance(cw))
    sv = np.linalg.svd(cw, compute_uv=False)
    assert np.allclose(lam, sv ** 2, rtol=1e-12, atol=1e-12 * sv[0] ** 2)


def test_windowed_covariance_is_weighted_sum_of_outer_products():
    # Eq. 12 brute force: sum over pixels of w_i^2 s_i^H s_i, one pixel at a time
    iq = _rand_packet(5, 4, 3, seed=5)
    win = O.window_boxes(4, 3, 2, 1, 1.0 / 3.0, 6.0)[0]
    w = O.window_table(win, 4, 3).reshape(-1)
    c = O.casorati(iq)
    ref = np.zeros((5, 5), dtype=complex)
    for i in range(c.shape[0]):
        s = c[i:i + 1, :]
        ref += w[i] ** 2 * (s.conj().T @ s)
    assert np.allclose(O.covariance(w[:, None] * c), ref, rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- EVD (Eq. 2)

def _circulant(lam):
    n = lam.shape[0]
    col = np.fft.ifft(lam)            # first column; eigenvalues of the circulant = fft(col) = lam
    idx = (np.arange(n)[:, None] - np.arange(n)[None, :]) % n
    return col[idx]


@pytest.mark.parametrize("nt", [32, 64, 100, 128, 200])
def test_evd_circulant_closed_form(nt):
    rng = np.random.default_rng(nt)
    lam = 10.0 ** rng.uniform(-8.0, 0.0, size=nt)
    r = _circulant(lam)
    assert np.allclose(r, r.conj().T, atol=1e-15)
    got, v = O.evd(r)
    assert np.allclose(got, np.sort(lam)[::-1], rtol=0, atol=1e-14)
    # eigenvector of the largest eigenvalue is a Fourier column
    j = int(np.argmax(lam))
    f = np.exp(2j * np.pi * np.arange(nt) * j / nt) / math.sqrt(nt)
    assert abs(abs(np.vdot(f, v[:, 0])) - 1.0) < 1e-10
    assert np.linalg.norm(v.conj().T @ v - np.eye(nt)) < 1e-12
    assert np.linalg.norm(r @ v - v * got[None, :]) < 1e-13 * np.linalg.norm(r)


def test_evd_rank_one_and_diagonal():
    rng = np.random.default_rng(7)
    z = rng.standard_normal(12) + 1j * rng.standard_normal(12)
    lam, v = O.evd(np.outer(z, z.conj()))
    assert abs(lam[0] - np.vdot(z, z).real) < 1e-12 * lam[0]
    assert np.all(np.abs(lam[1:]) < 1e-12 * lam[0])
    assert abs(abs(np.vdot(z / np.linalg.norm(z), v[:, 0])) - 1) < 1e-12
    d = np.array([3.0, 9.0, 1.0, 5.0])
    lam, v = O.evd(np.diag(d).astype(complex))
    assert np.array_equal(lam, np.array([9.0, 5.0, 3.0, 1.0]))


def test_evd_matches_plain_jacobi():
    rng = np.random.default_rng(8)
    for n in (4, 9, 16):
        x = rng.standard_normal((3 * n, n)) + 1j * rng.standard_normal((3 * n, n))
        r = x.conj().T @ x
        lam, v = O.evd(r)
        lam_j, v_j, _ = jacobi_eigh(r)
        assert np.allclose(lam, lam_j, rtol=1e-12)
        assert np.allclose(O.projector(v[:, :3], np.ones(3)),
                           O.projector(v_j[:, :3], np.ones(3)), atol=1e-10)


# ---------------------------------------------------------------- rules (Eqs 4, 6, 9)

def test_knee_hand_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "knee_hand.json")))
    lam = 10.0 ** np.array(g["log10_lambda"], dtype=np.float64)
    curv, flags = O.knee_curvature(lam, g["beta"])
    assert flags == 0
    assert np.allclose(curv, g["curvature"], atol=5e-7)
    assert O.knee_k(curv, 8, 0.5) == g["k_half"]
    assert O.knee_k(curv, 8, 1.0) == g["k_full"]
    w, k, _, _ = O.rule_weights(lam, O.Threshold(cut=O.CUT_KNEE, knee_max_frac=0.5))
    assert k == 4 and np.array_equal(w, [0, 0, 0, 0, 1, 1, 1, 1])


def test_knee_geometric_cliff_then_flat():
    # y = 9, 8, ..., 4 for n = 1..6, then flat at 4. Scaled by 32/9 the slope is
    # -3.556 per step. Worked by hand: y'(6) = -1.778, y'(7) = 0; y''(5,6,7) =
    # 0.889, 1.778, 0.889; K(5,6,7) = 0.0176, 0.2095, 0.889 -> k = 7, the first
    # flat point (low slope dominates the denominator of Eq. 6).
    nt = 32
    y = np.concatenate([-np.arange(0, 6, dtype=float), np.full(nt - 6, -5.0)]) + 9.0
    curv, _ = O.knee_curvature(10.0 ** y, 1.0)
    assert np.allclose(curv[4:7], [0.0176413, 0.2094885, 0.8888889], atol=1e-6)
    assert O.knee_k(curv, nt, 0.5) == 7


def test_knee_ties_take_smallest_index_and_scale():
    curv = np.array([0.0, 1.0, 0.5, 1.0, 0.2, 0.0, 0.0, 0.0])
    assert O.knee_k(curv, 8, 0.5) == 2
    # beta scales y'' and y' together: with beta -> 0 the curvature goes to |y''|*beta
    lam = 10.0 ** np.array([8, 6, 4, 2, 1.9, 1.8, 1.7, 1.6])
    c1, _ = O.knee_curvature(lam, 1e-6)
    c2, _ = O.knee_curvature(lam, 2e-6)
    assert np.allclose(c2, 2 * c1, rtol=1e-9)


def test_sigmoid_closed_form():
    w = O.sigmoid_weights(20, 7, 2.0)
    assert abs(w[6] - 0.5) < 1e-15                         # i = k
    assert np.allclose(w[6 + 3] + w[6 - 3], 1.0)           # symmetric about k
    assert abs(w[0] - 1.0 / (1.0 + math.exp(12.0))) < 1e-18
    assert np.all(np.diff(w) > 0)


def test_fixed_k_hard_and_soft():
    lam = np.linspace(10, 1, 10)
    w, k, _, _ = O.rule_weights(lam, O.Threshold(cut=O.CUT_FIXED_K, k_fixed=3))
    assert k == 3 and np.array_equal(w, [0, 0, 0] + [1] * 7)
    w, _, _, _ = O.rule_weights(lam, O.Threshold(cut=O.CUT_FIXED_K, k_fixed=3,
                                                 shape=O.SHAPE_SIGMOID, beta_sigmoid=2.0))
    assert abs(w[2] - 0.5) < 1e-15


def test_slope_rule_hand_worked():
    # lambda = 1, .5, .1, .09, .08, .07, .06, .05 (Nt = 8): y = 8 lambda / lambda_1 =
    # 8, 4, .8, .72, .64, .56, .48, .4; slopes (central inside, one-sided at the
    # ends) -4, -3.6, -1.64, -.08, -.08, -.08, -.08, -.08. Threshold 1.1: the first
    # slope with magnitude <= 1.1 is at 0-based n = 3, so k = 3; threshold 2 gives
    # k = 2 and threshold 5 gives k = 0. Forward differences would give k = 2 at
    # 1.1, the unscaled curve k = 0.
    lam = np.array([1.0, 0.5, 0.1, 0.09, 0.08, 0.07, 0.06, 0.05])
    assert O.slope_k(lam, 1.1) == (3, 0)
    assert O.slope_k(lam, 2.0) == (2, 0)
    assert O.slope_k(lam, 5.0) == (0, 0)
    w, k, _, _ = O.rule_weights(lam, O.Threshold(cut=O.CUT_SLOPE, slope_thr=1.1))
    assert k == 3 and np.array_equal(w, [0, 0, 0, 1, 1, 1, 1, 1])


def test_slope_rule_linear_spectrum_and_degenerate():
    # lambda_i = Nt - i scales to y = Nt - i exactly: every slope is -1, so a
    # threshold of 1 cuts nothing (|y'| <= 1 already at n = 0) and 0.5 cuts all
    nt = 16
    lam = np.arange(nt, 0, -1, dtype=np.float64)
    assert O.slope_k(lam, 1.0) == (0, 0)
    assert O.slope_k(lam, 0.5) == (nt, 0)
    w, k, _, flags = O.rule_weights(np.zeros(8), O.Threshold(cut=O.CUT_SLOPE))
    assert flags == 1 and k == 0 and np.all(w == 1)


def test_power_weights_flat_spectrum_is_the_window():
    # equal eigenvalues leave the window of Eq. 10 itself: for Nt = 5,
    # u_i = 2.5 i / 4 and win = exp(-u^2 / 2) = exp(0, -.1953125, -.78125,
    # -1.7578125, -3.125), already at maximum 1 for i = 0
    w, flags = O.power_weights(np.full(5, 3.0), 2.0)
    assert flags == 0
    assert np.allclose(w, np.exp([0.0, -0.1953125, -0.78125, -1.7578125, -3.125]), rtol=1e-14)


def test_power_weights_geometric_hand_worked():
    # lambda_i = 2^-i, Nt = 5, beta = 1: log wt_i = -.1953125 i^2 + i ln 2 =
    # 0, .4978347, .6050444, .3216290, -.3524113; the maximum is at i = 2
    w, _ = O.power_weights(2.0 ** -np.arange(5, dtype=np.float64), 1.0)
    lw = np.array([0.0, 0.4978347, 0.6050444, 0.3216290, -0.3524113])
    assert w[2] == 1.0
    assert np.allclose(w, np.exp(lw - lw[2]), rtol=1e-6)
    # a common scale of the eigenvalues cancels in the normalisation
    w2, _ = O.power_weights(7.5 * 2.0 ** -np.arange(5, dtype=np.float64), 1.0)
    assert np.allclose(w2, w, rtol=1e-13)


def test_power_weights_floor_and_degenerate():
    # zero eigenvalues are floored at lambda_1 2^-52: for Nt = 4 they dominate,
    # and the last one is worth win(3) / win(2) = exp(-(6.25 - 25 / 9) / 2)
    w, _ = O.power_weights(np.array([1.0, 0.5, 0.0, 0.0]), 1.0)
    assert w[2] == 1.0 and abs(w[3] - math.exp(-0.5 * (6.25 - 25.0 / 9.0))) < 1e-14
    assert w[0] < 1e-14
    w, k, _, flags = O.rule_weights(np.zeros(6), O.Threshold(cut=O.CUT_POWER))
    assert flags == 1 and k == -1 and np.all(w == 1)


def test_median_rule_geometric_odd_count():
    # Eq. 7 worked by hand: lambda_i = 2^-i, i = 0..8; the median is 2^-4. With
    # beta = 4 the threshold 1/4 equals lambda_2, which is kept (only eigenvalues
    # above it are tissue): k = 2. With beta = 3 the threshold 3/16 lies below
    # lambda_2: k = 3. A threshold divided by beta would give k = 9 and 6.
    lam = 2.0 ** -np.arange(9, dtype=np.float64)
    assert O.median_k(lam, 4.0) == 2
    assert O.median_k(lam, 3.0) == 3
    w, k, _, _ = O.rule_weights(lam, O.Threshold(cut=O.CUT_MEDIAN, beta_median=4.0))
    assert k == 2 and np.array_equal(w, [0, 0] + [1] * 7)


def test_median_rule_even_count_takes_mean_of_middle_pair():
    # lambda = 100, 10, 4, 2, 1, 0.5: the median of the even count is (4 + 2) / 2 = 3.
    # beta = 1: threshold 3, so 100, 10, 4 are tissue (k = 3); the lower middle
    # value as median would give threshold 4 and k = 2.
    # beta = 0.9: threshold 2.7, k = 3; the upper middle value would give 1.8 and k = 4.
    lam = np.array([100.0, 10.0, 4.0, 2.0, 1.0, 0.5])
    assert O.median_k(lam, 1.0) == 3
    assert O.median_k(lam, 0.9) == 3
    # the order of the input does not matter
    assert O.median_k(lam[::-1].copy(), 1.0) == 3


def test_median_rule_flat_spectrum_and_sigmoid():
    lam = np.full(7, 2.5)
    assert O.median_k(lam, 1.0) == 0          # nothing lies above its own median
    assert O.median_k(lam, 0.5) == 7
    w, k, _, _ = O.rule_weights(2.0 ** -np.arange(9, dtype=np.float64),
                                O.Threshold(cut=O.CUT_MEDIAN, beta_median=3.0, shape=O.SHAPE_SIGMOID,
                                            beta_sigmoid=2.0))
    assert k == 3 and abs(w[2] - 0.5) < 1e-15


def test_median_rule_above_spread_returns_input():
    # beta larger than lambda_1 / lambda_median rejects nothing: all-ones weights,
    # so the filter returns its input (Eqs 4, 11, 13)
    iq = synth.make_packet(synth.PacketSpec(24, 20, 12, 40.0, 0.3, ((10, 2, 0.4),), seed=9))[0]
    res = O.filter_packet(iq, 2, 2, O.Threshold(cut=O.CUT_MEDIAN, beta_median=1e12))
    assert all(k == 0 for k in res["k"])
    ref = iq.astype(np.complex128)
    assert np.linalg.norm(res["iq_out"] - ref) <= 1e-13 * np.linalg.norm(ref)


def test_knee_degenerate_spectrum_flagged():
    w, k, _, flags = O.rule_weights(np.zeros(8), O.Threshold(cut=O.CUT_KNEE))
    assert flags == 1 and k == 0 and np.all(w == 1)


# ---------------------------------------------------------------- projection + PD (Eqs 4, 5, 13)

def test_all_ones_weights_return_input():
    iq = synth.make_packet(synth.PacketSpec(24, 20, 12, 40.0, 0.3, ((10, 2, 0.4),), seed=9))[0]
    nd = 4
    thr = O.Threshold(cut=O.CUT_EXPLICIT, explicit_w=np.ones((nd, 12)))
    res = O.filter_packet(iq, 2, 2, thr)
    ref = iq.astype(np.complex128)
    assert np.linalg.norm(res["iq_out"] - ref) <= 1e-13 * np.linalg.norm(ref)


def test_global_flat_window_is_global_svd_filter():
    iq = _rand_packet(10, 8, 6, seed=10)
    k = 3
    res = O.filter_packet(iq, 1, 1, O.Threshold(cut=O.CUT_FIXED_K, k_fixed=k), sigma_frac=0.0)
    c = O.casorati(iq)
    u, s, vh = np.linalg.svd(c, full_matrices=False)
    chat = c - (u[:, :k] * s[:k]) @ vh[:k]
    got = O.casorati(res["iq_out"])
    assert np.linalg.norm(got - chat) <= 1e-12 * np.linalg.norm(chat)
    # PD of the single subset: alpha * sum_t |C_hat|^2 with alpha = Npix*Nt/||C_hat||^2
    e = np.sum(np.abs(chat) ** 2)
    pd = (8 * 6 * 10 / e) * np.sum(np.abs(chat) ** 2, axis=1)
    assert np.allclose(res["pd"].reshape(-1), pd, rtol=1e-11)


def test_each_subset_equals_bruteforce_svd_filter():
    iq = _rand_packet(8, 12, 10, seed=11)
    thr = O.Threshold(cut=O.CUT_KNEE, shape=O.SHAPE_SIGMOID, knee_max_frac=0.75)
    res = O.filter_packet(iq, 2, 2, thr, keep_chat=True)
    c = O.casorati(iq)
    for d, (rows, chat) in enumerate(res["chat"]):
        w = O.window_table(res["windows"][d], 12, 10).reshape(-1)[rows]
        cw = w[:, None] * c[rows]
        u, s, vh = np.linalg.svd(cw, full_matrices=False)
        ref = (u * (s * res["w"][d])[None, :]) @ vh
        assert np.linalg.norm(chat - ref) <= 1e-12 * np.linalg.norm(cw)
        # energy identity ||C_hat||^2 = sum_i w_i^2 lambda_i
        assert abs(np.sum(np.abs(chat) ** 2) - np.sum(res["w"][d] ** 2 * res["lam"][d])) \
            <= 1e-11 * np.sum(res["lam"][d])


def test_eq4_equals_eq5_and_one_hot_rank_one():
    iq = _rand_packet(8, 6, 6, seed=12)
    nd = 4
    ew = np.zeros((nd, 8))
    ew[:, 2] = 1.0
    res = O.filter_packet(iq, 2, 2, O.Threshold(cut=O.CUT_EXPLICIT, explicit_w=ew),
                          check_eq5=True, keep_chat=True)
    for d, (rows, chat) in enumerate(res["chat"]):
        s = np.linalg.svd(chat, compute_uv=False)
        assert s[1] <= 1e-12 * s[0]
        assert abs(s[0] ** 2 - res["lam"][d][2]) <= 1e-10 * res["lam"][d][2]


def test_frame_phase_invariance_needs_conjugate_transpose():
    iq = synth.make_packet(synth.spec_small(3))[0][:, :32, :32].copy()
    thr = O.Threshold(cut=O.CUT_KNEE, shape=O.SHAPE_SIGMOID)
    a = O.filter_packet(iq, 2, 2, thr)
    ph = np.exp(1j * np.random.default_rng(0).uniform(0, 2 * np.pi, size=32))
    iq2 = iq.astype(np.complex128) * ph[:, None, None]       # kept in complex128
    b = O.filter_packet(iq2, 2, 2, thr)
    for la, lb in zip(a["lam"], b["lam"]):
        assert np.allclose(la, lb, rtol=1e-9, atol=1e-12 * la[0])
    assert a["k"] == b["k"]
    assert np.allclose(a["pd"], b["pd"], rtol=1e-8)
    assert np.allclose(b["iq_out"], a["iq_out"] * ph[:, None, None],
                       atol=1e-8 * np.abs(a["iq_out"]).max())
    # a plain transpose (no conjugation) is not invariant: the covariance changes
    c = O.casorati(iq)
    c2 = O.casorati(iq2)
    assert np.allclose(O.covariance(c2), (ph.conj()[:, None] * O.covariance(c)) * ph[None, :])
    assert not np.allclose(np.linalg.eigvalsh(c2.T @ c2 + (c2.T @ c2).conj().T),
                           np.linalg.eigvalsh(c.T @ c + (c.T @ c).conj().T), rtol=1e-3)


def test_exact_rank_tissue_is_nulled():
    iq = _low_rank_packet(12, 10, 9, rank=3, dtype=np.complex128)    # exactly rank 3 in FP64
    res = O.filter_packet(iq, 2, 2, O.Threshold(cut=O.CUT_FIXED_K, k_fixed=3))
    assert np.linalg.norm(res["iq_out"]) <= 1e-12 * np.linalg.norm(iq)
    res = O.filter_packet(iq, 2, 2, O.Threshold(cut=O.CUT_FIXED_K, k_fixed=2))
    assert np.linalg.norm(res["iq_out"]) > 1e-3 * np.linalg.norm(iq)


def test_scale_behaviour_of_pd_modes():
    iq = _rand_packet(8, 10, 8, seed=13).astype(np.complex128)
    thr = O.Threshold(cut=O.CUT_FIXED_K, k_fixed=2)
    a = O.filter_packet(iq, 2, 2, thr)
    b = O.filter_packet(iq * 3.0, 2, 2, thr)
    assert np.allclose(a["pd"], b["pd"], rtol=1e-10)                     # Eq. 13 normalises
    thr_sum = O.Threshold(cut=O.CUT_FIXED_K, k_fixed=2, pd_mode=O.PD_SUM)
    a = O.filter_packet(iq, 2, 2, thr_sum)
    b = O.filter_packet(iq * (3.0 - 1.0j), 2, 2, thr_sum)
    assert np.allclose(b["pd"], 10.0 * a["pd"], rtol=1e-10)             # |3 - i|^2 = 10


def test_compensated_mode_divides_by_alpha_weighted_window_energy():
    iq = _rand_packet(8, 10, 8, seed=14)
    thr = O.Threshold(cut=O.CUT_FIXED_K, k_fixed=2)
    a = O.filter_packet(iq, 2, 2, thr)
    thr.pd_mode = O.PD_EQ13_COMPENSATED
    b = O.filter_packet(iq, 2, 2, thr)
    comp = np.zeros((10, 8))
    for d, win in enumerate(a["windows"]):
        comp += a["alpha"][d] * O.window_table(win, 10, 8) ** 2
    assert np.allclose(b["pd"], a["pd"] / comp, rtol=1e-12)


# ---------------------------------------------------------------- generator

def test_generator_powers():
    spec = synth.spec_clinical(0)
    iq, mask = synth.make_packet(spec)
    p_t = 10 * np.log10(np.mean(np.abs(iq[:, ~mask]) ** 2))
    p_b = 10 * np.log10(np.mean(np.abs(iq[:, mask]) ** 2))
    assert abs(p_t - 50.0) < 0.2
    assert abs(p_b - 10 * np.log10(1.1)) < 0.2        # blood 0 dB plus noise -10 dB
    spec0 = synth.PacketSpec(64, 64, 16, -300.0, 0.0, (), seed=5)
    iq0, _ = synth.make_packet(spec0)
    assert abs(10 * np.log10(np.mean(np.abs(iq0) ** 2)) + 10.0) < 0.2


# ------------------------------------------------------------------ method 4 (Eq. 8)

def _unitary(rng, n):
    q, r = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return q * (np.diag(r) / np.abs(np.diag(r)))[None, :]


def test_ncc_rule_hand_worked():
    """Eq. 8 on a constructed case whose |u_i| are known exactly (tests/golden/ncc_hand.json)."""
    g = json.load(open(os.path.join(GOLDEN, "ncc_hand.json")))
    h4 = np.array([[1, 1, 1, 1], [1, -1, 1, -1], [1, 1, -1, -1], [1, -1, -1, 1]], dtype=float) / 2.0
    u = np.zeros((8, 6), dtype=complex)
    u[0:4, 0:3] = h4[:, 0:3]
    u[4:8, 3:6] = h4[:, 0:3] * np.exp(1j * np.array([0.3, 1.1, 2.0]))[None, :]
    sig = np.array(g["sigma"], dtype=float)
    v = _unitary(np.random.default_rng(8), 6)
    c = (u * sig[None, :]) @ v.conj().T
    lam, vv = O.evd(O.covariance(c))
    curve = O.ncc_curve(c, lam, vv, fn=g["fn"])
    ref = np.array([np.nan if x is None else x for x in g["curve"]])
    assert np.array_equal(np.isnan(curve), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.allclose(curve[ok], ref[ok], atol=1e-12)
    k, fl = O.ncc_k(curve)
    assert (k, fl) == (g["k"], 0)


def test_ncc_rule_disjoint_supports_and_svd():
    """Tissue components on one half of the pixels, blood on the other: the
    curve is exactly 0 at the cut between the groups (fn = 5), and it equals the
    curve built from numpy's SVD left singular vectors."""
    rng = np.random.default_rng(9)
    npix, nt, ntis = 200, 20, 8
    ua, _ = np.linalg.qr(rng.standard_normal((100, ntis)) + 1j * rng.standard_normal((100, ntis)))
    ub, _ = np.linalg.qr(rng.standard_normal((100, nt - ntis)) + 1j * rng.standard_normal((100, nt - ntis)))
    u = np.zeros((npix, nt), dtype=complex)
    u[:100, :ntis] = ua
    u[100:, ntis:] = ub
    sig = np.sort(rng.uniform(1.0, 2.0, nt))[::-1] * np.r_[np.full(ntis, 100.0), np.ones(nt - ntis)]
    c = (u * sig[None, :]) @ _unitary(rng, nt).conj().T
    lam, v = O.evd(O.covariance(c))
    curve = O.ncc_curve(c, lam, v)
    assert abs(curve[ntis - 1]) <= 1e-12
    assert np.all(curve[[i for i in range(O.NCC_FN - 1, nt - O.NCC_FN) if i != ntis - 1]] > 1e-3)
    assert O.ncc_k(curve) == (ntis, 0)
    # the same curve from the SVD's left singular vectors (Eq. 3, C = U D V^H)
    us, s, _ = np.linalg.svd(c, full_matrices=False)
    a = np.abs(us)
    ref = np.full(nt, np.nan)
    for k in range(O.NCC_FN, nt - O.NCC_FN + 1):
        it, ib = a[:, k - O.NCC_FN:k].sum(1), a[:, k:k + O.NCC_FN].sum(1)
        ref[k - 1] = it @ ib / np.sqrt((it @ it) * (ib @ ib))
    ok = ~np.isnan(ref)
    assert np.array_equal(np.isnan(curve), ~ok) and np.allclose(curve[ok], ref[ok], atol=1e-10)


def test_ncc_rule_shapes_and_degenerate():
    """Method 5 is the sigmoid of Eq. 9 centred on the Eq. 8 cut; a spectrum
    with no valid k (an all-zero subset) keeps every component and is flagged."""
    curve = np.full(16, np.nan)
    curve[4:11] = [0.9, 0.5, 0.2, 0.2, 0.6, 0.7, 0.8]
    lam = np.geomspace(1e6, 1.0, 16)
    w, k, cv, fl = O.rule_weights(lam, O.Threshold(cut=O.CUT_NCC, shape=O.SHAPE_SIGMOID, beta_sigmoid=2.0),
                                  ncc=curve)
    assert k == 7 and fl == 0                       # first of the two equal minima
    assert np.allclose(w, O.sigmoid_weights(16, 7, 2.0), atol=0)
    w, k, _, _ = O.rule_weights(lam, O.Threshold(cut=O.CUT_NCC, shape=O.SHAPE_HARD), ncc=curve)
    assert np.array_equal(w, (np.arange(1, 17) > 7).astype(float))
    z = np.zeros((30, 12), dtype=complex)
    lam0, v0 = O.evd(O.covariance(z))
    c0 = O.ncc_curve(z, lam0, v0)
    assert np.all(np.isnan(c0)) and O.ncc_k(c0) == (0, O.lcf_oracle.FLAG_NONPOSITIVE)


def test_sliding_packets_share_covariance_block():
    """Consecutive sliding packets (hop h) share every frame pair but the new
    ones: R_{p+1}[:nt-h, :nt-h] = R_p[h:, h:] for every window (Eq. 12 sums
    over the same pixels and frame pairs), the identity an incremental
    covariance update relies on; the last h rows and columns are new."""
    import synth
    nt, hop = 20, 4
    spec = synth.PacketSpec(24, 20, nt + 3 * hop, 50.0, 0.4, ((8, 2, 0.6),), seed=11)
    rec, _ = synth.make_packet(spec)
    res = O.filter_stream(rec, nt, hop, 2, 2, O.Threshold(cut=O.CUT_FIXED_K, k_fixed=2))
    assert len(res) == 4
    for p in range(3):
        for d in range(4):
            a, b = res[p]["cov"][d], res[p + 1]["cov"][d]
            assert np.allclose(b[:nt - hop, :nt - hop], a[hop:, hop:], rtol=1e-12, atol=1e-12 * abs(a[0, 0]))
            # the new frames do change the rest
            assert not np.allclose(b[nt - hop:, :], a[nt - hop:, :])


def test_mlp_gate_hand_worked_and_invariances():
    """Gate statistic of two weight sets: hand-worked two-component case, zero
    for equal or proportional weights (Eq. 13 normalises the filtered energy),
    +inf when only one set keeps a component."""
    lam = np.array([4.0, 1.0])
    # shares p = [0.16, 1] / 1.16, q = [0.04, 1] / 1.04
    g = O.mlp_gate(lam, np.array([0.1, 1.0]), np.array([0.2, 1.0]))
    p0, q0 = 0.16 / 1.16, 0.04 / 1.04
    assert abs(g - abs(10 * np.log10(q0 / p0))) < 1e-12
    assert abs(g - 5.5464) < 1e-4
    w = np.array([0.3, 0.9, 1.0, 0.2])
    l4 = np.array([10.0, 3.0, 1.0, 0.5])
    assert O.mlp_gate(l4, w, w) == 0.0
    assert abs(O.mlp_gate(l4, 0.37 * w, w)) < 1e-12
    assert O.mlp_gate(lam, np.array([0.5, 1.0]), np.array([0.0, 1.0])) == np.inf
    # a component below the share in both sets is ignored
    assert O.mlp_gate(np.array([1e-6, 1.0]), np.array([1.0, 1.0]), np.array([0.5, 1.0])) < 1e-5


def test_mlp_gate_bounds_recombined_power_doppler():
    """With no share cut the gate is a bound: on a small windowed packet, the
    Eq. 13 power Doppler of the filter with one weight set differs from the
    other's by at most the gate's largest subset value, at every pixel."""
    rng = np.random.default_rng(5)
    nt, ny, nx = 10, 9, 8
    iq = (rng.standard_normal((nt, ny, nx)) + 1j * rng.standard_normal((nt, ny, nx))).astype(np.complex64)
    w_rule = np.tile(O.sigmoid_weights(nt, 3, 2.0), (4, 1))
    w_net = np.clip(w_rule + 0.2 * rng.standard_normal(w_rule.shape), 0.05, 1.0)
    ra = O.filter_packet(iq, 2, 2, O.Threshold(cut=O.CUT_EXPLICIT, explicit_w=w_rule))
    rb = O.filter_packet(iq, 2, 2, O.Threshold(cut=O.CUT_EXPLICIT, explicit_w=w_net))
    g = max(O.mlp_gate(ra["lam"][d], w_net[d], w_rule[d], share=0.0) for d in range(4))
    dev = np.abs(10 * np.log10(rb["pd"] / ra["pd"]))
    assert 0.0 < dev.max() <= g + 1e-9
