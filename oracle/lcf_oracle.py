"""Plain FP64 reference of the localized EVD clutter filter (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use this module. It is slow on purpose: every step is the
definition written out with numpy / LAPACK, in complex128, in the paper's
order:

1. Casorati matrix C (pixels x frames) of the packet   -- Principles section, Fig. 1
2. Gaussian windows, C_w = W C                          -- Eq. 11
3. Covariance R = C_w^H C_w                             -- Eqs 1 and 12
4. EVD R = V Lambda V^H, eigenvalues descending         -- Eq. 2
5. Eigencomponent weights (hard / curvature / slope / median / sigmoid /
   eigenvalue power)                                   -- Eqs 4, 6, 7, 9, 10, Fig. 2c
6. Projection C_hat = C_w V diag(w) V^H                 -- Eqs 4 and 5
7. Power Doppler PD_d = sum_t |C_hat|^2                 -- text after Eq. 5
8. Recombination PD = sum_d alpha_d PD_d, alpha_d = 1/(mean flow power)  -- Eq. 13

Readings where the paper is silent or ambiguous:
transposes of complex data are conjugate transposes; PD integrates (sums) over
slow time; the mean flow power of a subset is taken over all Npix pixels and
Nt frames, so alpha_d = Npix*Nt / sum_i w_i^2 lambda_i; window centres sit at
(j + 1/2)*spacing - 1/2 with sigma = sigma_frac * spacing and the window is
zero outside a +-trunc_sigmas*sigma box; the curvature rule takes numpy-style
differences (central inside, one-sided at the ends), searches
n in [2, floor(knee_max_frac*Nt)] and keeps the smallest index on ties; k is
the number of rejected leading components; the median rule takes the mean of
the two middle eigenvalues when Nt is even and rejects only eigenvalues strictly
above its threshold; the slope rule differentiates y(n) = lambda_n scaled as the
curvature rule scales its curve (Nt y(n) / y(1)) and cuts before the first n
whose slope magnitude is at most its threshold; the window of Eq. 10 is the half
of a Gaussian window of length 2 Nt - 1 with MATLAB's default width (alpha 2.5)
that starts at its peak, eigenvalues are floored at lambda_1 2^-52 there, and
"normalised" scales the weights to a maximum of 1; the combined filtered IQ is
sum_d C_hat_d / sum_d w_d. Method 4 (Eq. 8) takes the left singular vectors
u_i = C_w v_i / sigma_i of the windowed subset (u_i = 0 where sigma_i = 0), the
images I_T(k) = sum of |u_i| over i = k-fn+1..k and I_B(k) = over i = k+1..k+fn
(fn = 5, unit weights), their normalised cross-correlation as Eq. 8 writes it
(no mean removed), over 1-based k in [fn, Nt - fn] where both sums exist, and k
= the smallest index of the minimum; a pair of zero images gives no value there.
"""
from __future__ import annotations

from dataclasses import dataclass
import math
from typing import Optional

import numpy as np

CUT_FIXED_K, CUT_KNEE, CUT_EXPLICIT, CUT_MLP, CUT_MEDIAN, CUT_SLOPE, CUT_POWER, CUT_NCC = 0, 1, 2, 3, 4, 5, 6, 7
NCC_FN = 5     # singular vectors on each side of the cut (method 4: fn = 5)
SHAPE_HARD, SHAPE_SIGMOID = 0, 1
PD_EQ13, PD_SUM, PD_EQ13_COMPENSATED = 0, 1, 2

FLAG_NONPOSITIVE = 1 << 0   # lambda_1 <= 0 or log10(lambda_1) == 0 under the curvature rule
FLAG_MLP_FALLBACK = 1 << 3  # learned weights rejected: the rule's weights are used
GATE_SHARE = 1e-3           # components below this share of both filtered energies are ignored


@dataclass
class Threshold:
    """Thresholding rule (mirrors the C struct ``lcf_threshold``)."""
    cut: int = CUT_FIXED_K
    shape: int = SHAPE_HARD
    pd_mode: int = PD_EQ13
    k_fixed: int = 4
    beta_knee: float = 1.0
    knee_max_frac: float = 0.5
    beta_sigmoid: float = 2.0
    beta_median: float = 1.43                   # Eq. 7 scaling factor (Fig. 2a's example)
    slope_thr: float = 1.1                      # slope rule threshold (Fig. 2c's example)
    beta_power: float = 2.0                     # Eq. 10 order (Fig. 2g's example)
    explicit_w: Optional[np.ndarray] = None     # [nd][nt]
    mlp: Optional[object] = None                # callable(lam) -> weights, for CUT_MLP
    mlp_gate_db: Optional[float] = None         # CUT_MLP: gate threshold (dB); None = no gate


@dataclass
class Window:
    cy: float
    cx: float
    sy: float
    sx: float
    y0: int
    y1: int
    x0: int
    x1: int
    flat: bool


def window_boxes(ny: int, nx: int, gy: int, gx: int, sigma_frac: float = 1.0 / 3.0,
                 trunc_sigmas: float = 6.0):
    """Window grid of Eq. 11 / Fig. 3: gy x gx Gaussian windows, subset index
    d = a*gx + b. Centres (j + 1/2)*spacing - 1/2, sigma = sigma_frac*spacing
    per axis (the paper leaves both to the number of subsets). sigma_frac == 0
    gives one flat window over the whole image (global processing)."""
    out = []
    dy, dx = ny / gy, nx / gx
    for a in range(gy):
        for b in range(gx):
            cy = (a + 0.5) * dy - 0.5
            cx = (b + 0.5) * dx - 0.5
            sy = sigma_frac * dy
            sx = sigma_frac * dx
            flat = sigma_frac == 0.0
            if flat or trunc_sigmas == 0.0:
                y0, y1, x0, x1 = 0, ny - 1, 0, nx - 1
            else:
                y0 = max(0, int(math.ceil(cy - trunc_sigmas * sy)))
                y1 = min(ny - 1, int(math.floor(cy + trunc_sigmas * sy)))
                x0 = max(0, int(math.ceil(cx - trunc_sigmas * sx)))
                x1 = min(nx - 1, int(math.floor(cx + trunc_sigmas * sx)))
            out.append(Window(cy, cx, sy, sx, y0, y1, x0, x1, flat))
    return out


def window_table(win: Window, ny: int, nx: int) -> np.ndarray:
    """Full-image weights w_d(y, x) of one window (Eq. 11), zero outside its box."""
    w = np.zeros((ny, nx))
    ys = np.arange(win.y0, win.y1 + 1, dtype=np.float64)
    xs = np.arange(win.x0, win.x1 + 1, dtype=np.float64)
    if win.flat:
        w[win.y0:win.y1 + 1, win.x0:win.x1 + 1] = 1.0
    else:
        wy = np.exp(-((ys - win.cy) ** 2) / (2.0 * win.sy ** 2))
        wx = np.exp(-((xs - win.cx) ** 2) / (2.0 * win.sx ** 2))
        w[win.y0:win.y1 + 1, win.x0:win.x1 + 1] = np.outer(wy, wx)
    return w


def casorati(iq: np.ndarray) -> np.ndarray:
    """Casorati matrix of a packet (Fig. 1): rows = pixels (y-major), columns =
    frames. ``iq`` is [nt][ny][nx]; complex64 widens to complex128 exactly."""
    nt = iq.shape[0]
    return np.asarray(iq, dtype=np.complex128).reshape(nt, -1).T.copy()


def covariance(cw: np.ndarray) -> np.ndarray:
    """Temporal covariance R = C_w^H C_w (Eqs 1 and 12, conjugate transpose)."""
    return cw.conj().T @ cw


def evd(r: np.ndarray):
    """Eigen-decomposition R = V diag(lam) V^H (Eq. 2), eigenvalues descending."""
    lam, v = np.linalg.eigh(r)
    return lam[::-1].copy(), v[:, ::-1].copy()


def knee_curvature(lam: np.ndarray, beta: float):
    """Curvature of the normalised log-eigenvalue curve (Eq. 6).

    y(n) = log10(lambda_n) with lambda floored at lambda_1 * 2^-52, normalised
    to beta * Nt * y(n) / y(1); first and second derivatives by numpy-style
    differences; K = |y''| / (1 + y'^2)^(3/2). Returns (K, flags)."""
    nt = lam.shape[0]
    lam1 = lam[0]
    if not lam1 > 0.0:
        return np.zeros(nt), FLAG_NONPOSITIVE
    lamc = np.maximum(lam, lam1 * 2.0 ** -52)
    y = np.log10(lamc)
    if y[0] == 0.0:
        return np.zeros(nt), FLAG_NONPOSITIVE
    yt = beta * nt * y / y[0]
    d1 = np.gradient(yt)
    d2 = np.gradient(d1)
    return np.abs(d2) / (1.0 + d1 * d1) ** 1.5, 0


def knee_k(curv: np.ndarray, nt: int, max_frac: float) -> int:
    """k = smallest argmax of the curvature over 1-based n in [2, floor(max_frac*Nt)]."""
    hi = max(2, int(math.floor(max_frac * nt)))
    hi = min(hi, nt)
    seg = curv[1:hi]          # 0-based indices 1..hi-1  <=>  1-based n = 2..hi
    return int(np.argmax(seg)) + 2


def slope_k(lam: np.ndarray, thr: float):
    """Method 2 (the slope rule, Fig. 2c): the eigenvalue curve y(n) = lambda_n,
    scaled as the curvature rule scales its curve, y(n) Nt / y(1); its first
    derivative by central differences inside and one-sided ones at the ends; the
    leading components are tissue up to the turning point, the first n whose
    slope magnitude is at most ``thr``. Returns (k, flags): k = that 0-based n
    (Nt when every slope is steeper); lambda_1 <= 0 gives k = 0 and NONPOSITIVE."""
    lam = np.asarray(lam, dtype=np.float64)
    nt = lam.shape[0]
    if not lam[0] > 0.0:
        return 0, FLAG_NONPOSITIVE
    y = nt * lam / lam[0]
    for n in range(nt):
        if n == 0:
            d = y[1] - y[0]
        elif n == nt - 1:
            d = y[nt - 1] - y[nt - 2]
        else:
            d = 0.5 * (y[n + 1] - y[n - 1])
        if abs(d) <= thr:
            return n, 0
    return nt, 0


def power_weights(lam: np.ndarray, beta: float):
    """Method 6 (Eq. 10 with its Gaussian window): wt_i = win(i) / lambda_i^beta,
    i = 0..Nt-1, win(i) = exp(-(2.5 i / (Nt - 1))^2 / 2), then wt / max(wt).
    Eigenvalues are floored at lambda_1 2^-52. Returns (w, flags); lambda_1 <= 0
    gives all-ones weights and NONPOSITIVE."""
    lam = np.asarray(lam, dtype=np.float64)
    nt = lam.shape[0]
    if not lam[0] > 0.0:
        return np.ones(nt), FLAG_NONPOSITIVE
    lf = np.maximum(lam, lam[0] * 2.0 ** -52)
    i = np.arange(nt, dtype=np.float64)
    win = np.exp(-0.5 * (2.5 * i / (nt - 1)) ** 2)
    wt = win / lf ** beta
    return wt / np.max(wt), 0


def median_k(lam: np.ndarray, beta: float) -> int:
    """Method 3 (Eq. 7): threshold T = beta * lambda_median; the components whose
    eigenvalue exceeds T are tissue, so k = #{i : lambda_i > T}. The median of an
    even number of eigenvalues is the mean of the two middle ones."""
    s = np.sort(np.asarray(lam, dtype=np.float64))[::-1]
    n = s.shape[0]
    h = n // 2
    med = s[h] if n % 2 == 1 else 0.5 * (s[h - 1] + s[h])
    t = beta * med
    return int(np.count_nonzero(s > t))


def ncc_curve(cw: np.ndarray, lam: np.ndarray, v: np.ndarray, fn: int = NCC_FN) -> np.ndarray:
    """Method 4 (Eq. 8): normalised cross-correlation of the tissue image
    I_T(k) = sum_{i=k-fn+1..k} |u_i| and the blood image I_B(k) = sum_{i=k+1..k+fn} |u_i|,
    with the left singular vectors u_i = C_w v_i / sigma_i, sigma_i^2 = lambda_i
    (C V = U D). Entry k-1 holds 1-based k in [fn, Nt - fn]; NaN elsewhere and
    where an image is zero."""
    lam = np.asarray(lam, dtype=np.float64)
    nt = lam.shape[0]
    sig = np.sqrt(np.maximum(lam, 0.0))
    u = cw @ v
    inv = np.where(sig > 0.0, 1.0 / np.where(sig > 0.0, sig, 1.0), 0.0)
    a = np.abs(u) * inv[None, :]
    curve = np.full(nt, np.nan)
    for k in range(fn, nt - fn + 1):
        it = a[:, k - fn:k].sum(axis=1)
        ib = a[:, k:k + fn].sum(axis=1)
        den = math.sqrt(float(it @ it)) * math.sqrt(float(ib @ ib))
        if den > 0.0:
            curve[k - 1] = float(it @ ib) / den
    return curve


def ncc_k(curve: np.ndarray):
    """k = the smallest 1-based index of the minimum of Eq. 8's curve; 0 and the
    NONPOSITIVE flag when no k has a value."""
    if not np.any(np.isfinite(curve)):
        return 0, FLAG_NONPOSITIVE
    c = np.where(np.isfinite(curve), curve, np.inf)
    return int(np.argmin(c)) + 1, 0


def sigmoid_weights(nt: int, k: int, beta: float) -> np.ndarray:
    """Soft weights of Eq. 9: w_i = 1 / (1 + exp(-beta (i - k))), i = 1..Nt."""
    i = np.arange(1, nt + 1, dtype=np.float64)
    return 1.0 / (1.0 + np.exp(-beta * (i - k)))


def rule_weights(lam: np.ndarray, thr: Threshold, d: int = 0, ncc=None):
    """Eigencomponent weights of one subset.

    FIXED_K / KNEE / MEDIAN / SLOPE / NCC choose k (Eq. 4 hard cut, Eq. 6
    curvature, Eq. 7 median, the slope rule of Fig. 2c, Eq. 8 with its curve
    ``ncc`` from ``ncc_curve``); the shape is a hard 0/1 cut (Eq. 4) or the
    sigmoid of Eq. 9 centred on k (method 5 with the NCC cut). EXPLICIT takes
    the caller's weights; MLP calls ``thr.mlp(lam)``. Returns (w, k, curv, flags);
    curv is the Eq. 6 or Eq. 8 curve where the rule has one."""
    nt = lam.shape[0]
    curv = np.zeros(nt)
    flags = 0
    if thr.cut == CUT_EXPLICIT:
        return np.asarray(thr.explicit_w[d], dtype=np.float64).copy(), -1, curv, 0
    if thr.cut == CUT_MLP:
        w = np.asarray(thr.mlp(lam), dtype=np.float64)
        if thr.mlp_gate_db is None:
            return w, -1, curv, 0
        # the plain rule (curvature cut with the threshold's shape) is the fallback
        rule = Threshold(cut=CUT_KNEE, shape=thr.shape, beta_knee=thr.beta_knee,
                         knee_max_frac=thr.knee_max_frac, beta_sigmoid=thr.beta_sigmoid)
        w_rule, k, curv, flags = rule_weights(lam, rule)
        if mlp_gate(lam, w, w_rule) < thr.mlp_gate_db:
            return w, -1, curv, flags
        return w_rule, k, curv, flags | FLAG_MLP_FALLBACK
    if thr.cut == CUT_POWER:
        w, flags = power_weights(lam, thr.beta_power)
        return w, -1, curv, flags
    if thr.cut == CUT_FIXED_K:
        k = int(thr.k_fixed)
    elif thr.cut == CUT_KNEE:
        curv, flags = knee_curvature(lam, thr.beta_knee)
        k = 0 if flags else knee_k(curv, nt, thr.knee_max_frac)
    elif thr.cut == CUT_MEDIAN:
        k = median_k(lam, thr.beta_median)
    elif thr.cut == CUT_SLOPE:
        k, flags = slope_k(lam, thr.slope_thr)
    elif thr.cut == CUT_NCC:
        curv = np.asarray(ncc, dtype=np.float64)
        k, flags = ncc_k(curv)
    else:
        raise ValueError("unknown cut")
    if thr.shape == SHAPE_HARD:
        w = (np.arange(1, nt + 1) > k).astype(np.float64)
    else:
        w = sigmoid_weights(nt, k, thr.beta_sigmoid)
    return w, k, curv, flags


def mlp_gate(lam: np.ndarray, w_net: np.ndarray, w_rule: np.ndarray, share: float = GATE_SHARE) -> float:
    """Predicted power Doppler deviation (dB) between two weight sets of one
    subset. After Eq. 13 the subset's power Doppler at a pixel is proportional
    to sum_i q_i e_i(x), with q_i = w_i^2 lambda_i / sum_j w_j^2 lambda_j and
    e_i(x) = |(C_w v_i)(x)|^2 / lambda_i shared by both sets, so the ratio of the
    two images at a pixel lies between the extreme ratios q_i(net) / q_i(rule)
    of the components present there. Returned: the largest |10 log10| of that
    ratio over the components (lambda_i > 0) holding at least ``share`` of
    either filtered energy; +inf if only one set keeps such a component or an
    energy is zero."""
    lam = np.asarray(lam, dtype=np.float64)
    en = np.asarray(w_net, dtype=np.float64) ** 2 * lam
    er = np.asarray(w_rule, dtype=np.float64) ** 2 * lam
    tn, tr = float(np.sum(en)), float(np.sum(er))
    if not (tn > 0.0 and tr > 0.0):
        return math.inf
    g = 0.0
    for i in range(lam.shape[0]):
        if not lam[i] > 0.0:
            continue
        q, p = en[i] / tn, er[i] / tr
        if q >= share or p >= share:
            g = max(g, abs(10.0 * math.log10(q / p)) if (q > 0.0 and p > 0.0) else math.inf)
    return g


def projector(v: np.ndarray, w: np.ndarray) -> np.ndarray:
    """P = V diag(w) V^H (Eq. 4 with Lambda_hat = diag(w))."""
    return (v * w[None, :]) @ v.conj().T


def filter_packet(iq: np.ndarray, gy: int, gx: int, thr: Threshold,
                  sigma_frac: float = 1.0 / 3.0, trunc_sigmas: float = 6.0,
                  check_eq5: bool = False, keep_chat: bool = False, subsets=None):
    """Localized EVD clutter filter of one packet (Eqs 11-13).

    Returns a dict with ``iq_out`` ([nt][ny][nx] complex128), ``pd`` ([ny][nx]),
    and per-subset ``lam``, ``v``, ``w``, ``k``, ``curv``, ``alpha``, ``flags``,
    ``cov`` and ``wsum`` (sum_d w_d). ``subsets`` (a list of subset indices)
    restricts the work to those windows (a timing sample; the recombined
    outputs then cover those windows only)."""
    nt, ny, nx = iq.shape
    npix = ny * nx
    cfull = casorati(iq)                                   # [npix][nt]
    wins = window_boxes(ny, nx, gy, gx, sigma_frac, trunc_sigmas)
    nd = len(wins)
    acc = np.zeros((npix, nt), dtype=np.complex128)
    wsum = np.zeros(npix)
    pd_parts = []
    res = dict(lam=[], v=[], w=[], k=[], curv=[], alpha=[], flags=[], cov=[], chat=[])
    for d, win in enumerate(wins):
        if subsets is not None and d not in subsets:
            continue
        wfull = window_table(win, ny, nx).reshape(-1)
        rows = (np.arange(win.y0, win.y1 + 1)[:, None] * nx
                + np.arange(win.x0, win.x1 + 1)[None, :]).reshape(-1)
        wv = wfull[rows]
        cw = wv[:, None] * cfull[rows]                         # Eq. 11
        r = covariance(cw)                                     # Eq. 12
        lam, v = evd(r)                                        # Eq. 2
        ncc = ncc_curve(cw, lam, v) if thr.cut == CUT_NCC else None   # Eq. 8
        w, k, curv, flags = rule_weights(lam, thr, d, ncc)
        p = projector(v, w)
        chat = cw @ p                                          # Eq. 4
        if check_eq5:
            chat5 = cw @ (np.eye(nt) - projector(v, 1.0 - w))  # Eq. 5
            assert np.allclose(chat, chat5, rtol=1e-9, atol=1e-9 * np.linalg.norm(cw))
        energy = float(np.sum(np.abs(chat) ** 2))
        if thr.pd_mode == PD_SUM:
            alpha = 1.0
        else:
            alpha = npix * nt / energy if energy > 0.0 else 0.0   # Eq. 13
        pdd = np.sum(np.abs(chat) ** 2, axis=1)
        pd_parts.append((rows, pdd, alpha, wv))
        acc[rows] += chat
        wsum[rows] += wv
        for key, val in (("lam", lam), ("v", v), ("w", w), ("k", k), ("curv", curv),
                         ("alpha", alpha), ("flags", flags), ("cov", r)):
            res[key].append(val)
        if keep_chat:
            res["chat"].append((rows, chat))
    pd = np.zeros(npix)
    comp = np.zeros(npix)
    for rows, pdd, alpha, wv in pd_parts:
        pd[rows] += alpha * pdd
        comp[rows] += alpha * wv * wv
    if thr.pd_mode == PD_EQ13_COMPENSATED:
        pd = np.where(comp > 0.0, pd / np.where(comp > 0.0, comp, 1.0), 0.0)
    out = np.where(wsum[:, None] > 0.0, acc / np.where(wsum > 0.0, wsum, 1.0)[:, None], 0.0)
    res["iq_out"] = out.T.reshape(nt, ny, nx)
    res["pd"] = pd.reshape(ny, nx)
    res["wsum"] = wsum.reshape(ny, nx)
    res["nd"] = nd
    res["windows"] = wins
    return res


def filter_stream(record: np.ndarray, nt: int, hop: int, gy: int, gx: int, thr: Threshold,
                  count: int = None, **kw):
    """Sliding packets of a recording (the Experimental Studies section times the
    filter over packets that slide by a few frames): packet p holds frames
    [p hop, p hop + nt) of ``record`` ([T][ny][nx]) and is filtered from scratch
    by ``filter_packet``. Returns the list of per-packet results."""
    total = record.shape[0]
    n = (total - nt) // hop + 1
    if count is not None:
        n = min(n, count)
    return [filter_packet(record[p * hop:p * hop + nt], gy, gx, thr, **kw) for p in range(n)]

