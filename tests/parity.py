"""Comparison helpers for GPU-vs-oracle parity (test infrastructure)."""
import sys

import numpy as np

import oracle as O


def rel_fro(a, b) -> float:
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def dilate(mask: np.ndarray, r: int) -> np.ndarray:
    out = mask.copy()
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            out |= np.roll(np.roll(mask, dy, axis=0), dx, axis=1)
    return out


def pd_db_error(pd_gpu, pd_or, tube_mask):
    """Max / p99 / p99.9 of |10 log10(PD_gpu / PD_oracle)| over pixels above the
    noise floor: floor = median oracle PD outside the vessels dilated by 2 px,
    'above' = PD_oracle >= 2 x floor."""
    pd_or = np.asarray(pd_or, dtype=np.float64)
    pd_gpu = np.asarray(pd_gpu, dtype=np.float64)
    bg = ~dilate(tube_mask, 2)
    floor = np.median(pd_or[bg]) if np.any(bg) else np.median(pd_or)
    sel = pd_or >= 2.0 * floor
    err = np.abs(10.0 * np.log10(np.maximum(pd_gpu[sel], 1e-300) / pd_or[sel]))
    if err.size == 0:
        return 0.0, 0.0, 0.0, 0
    return float(err.max()), float(np.percentile(err, 99)), float(np.percentile(err, 99.9)), int(sel.sum())


def knee_tie(curv: np.ndarray, k_a: int, k_b: int, rtol: float = 1e-9) -> bool:
    """Two cut indices are a tie when the curvature at both agrees within rtol."""
    a, b = curv[k_a - 1], curv[k_b - 1]
    return abs(a - b) <= rtol * max(abs(a), abs(b))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_gpu(lcf, ctx, iq_np, gy, gx, thr, **kw):
    import torch
    iq = torch.from_numpy(iq_np).cuda()
    io, pd, dg = ctx.filter(iq, gy, gx, thr, diag=True, **kw)
    torch.cuda.synchronize()
    st = ctx.sync()
    assert st == 0, f"lcf_sync status {st}"
    d = {k: v.cpu().numpy() for k, v in dg.items()}
    return (io.cpu().numpy() if io is not None else None), pd.cpu().numpy(), d


def oracle_thr(lcf_thr, nd=None, explicit=None):
    return O.Threshold(cut=lcf_thr.cut, shape=lcf_thr.shape, pd_mode=lcf_thr.pd_mode, k_fixed=lcf_thr.k_fixed,
                       beta_knee=lcf_thr.beta_knee, knee_max_frac=lcf_thr.knee_max_frac,
                       beta_sigmoid=lcf_thr.beta_sigmoid, beta_median=lcf_thr.beta_median,
                       slope_thr=lcf_thr.slope_thr, beta_power=lcf_thr.beta_power, explicit_w=explicit)


def slope_tie(lam, thr, k1, k2):
    """True when the slope at the earlier of two turning points lies within the
    eigenvalue parity tolerance of the slope rule's threshold on ``lam``."""
    lam = np.asarray(lam, dtype=np.float64)
    nt = lam.shape[0]
    y = nt * lam / lam[0]
    n = min(k1, k2)
    d = y[1] - y[0] if n == 0 else (y[n] - y[n - 1] if n == nt - 1 else 0.5 * (y[n + 1] - y[n - 1]))
    return abs(abs(d) - thr) <= 1e-4 * thr + 1e-6 * nt


def median_tie(lam, beta, k1, k2):
    """True when every eigenvalue between the two cuts lies within the eigenvalue
    parity tolerance of the median rule's threshold (Eq. 7) on ``lam``."""
    s = np.sort(np.asarray(lam, dtype=np.float64))[::-1]
    n, h = s.shape[0], s.shape[0] // 2
    t = beta * (s[h] if n % 2 else 0.5 * (s[h - 1] + s[h]))
    lo, hi = min(k1, k2), max(k1, k2)
    return all(abs(s[i] - t) <= 1e-5 * t + 1e-7 * s[0] for i in range(lo, hi))


def check_end_to_end(lcf, ctx, iq, mask, gy, gx, thr, tol_fro, tol_db, name, precision=0,
                     sigma_frac=1.0 / 3.0, trunc_sigmas=6.0):
    say(f"[{name}] shape={iq.shape} grid={gy}x{gx} cut={thr.cut} shape={thr.shape} pd_mode={thr.pd_mode} "
        f"trunc={trunc_sigmas} prec={precision}")
    geo = dict(sigma_frac=sigma_frac, trunc_sigmas=trunc_sigmas)
    io, pd, d = run_gpu(lcf, ctx, iq, gy, gx, thr, precision=precision, **geo)
    e_fro, emax = compare_with_oracle(lcf, iq, mask, gy, gx, thr, io, pd, d, tol_fro, tol_db, **geo)
    return e_fro, emax, io, pd


def compare_with_oracle(lcf, iq, mask, gy, gx, thr, io, pd, d, tol_fro, tol_db, res=None, **geo):
    """Decision and numeric parity of one packet's GPU outputs (io, pd, diag d)
    with the oracle (``res``: its filter_packet result, computed if None)."""
    if res is None:
        res = O.filter_packet(iq, gy, gx, oracle_thr(thr), **geo)
    nd = gy * gx
    # decision parity: the oracle's FP64 rule on the GPU's eigenvalues
    forced = False
    for s in range(nd):
        lam_g = d["eigvals"][s]
        lam_o = res["lam"][s]
        assert np.allclose(lam_g, lam_o, rtol=1e-5, atol=1e-7 * lam_o[0]), (s, np.max(np.abs(lam_g - lam_o) / lam_o[0]))
        if thr.cut == lcf.CUT_POWER:
            w_rule, _, _, _ = O.rule_weights(lam_g, oracle_thr(thr))
            assert np.allclose(d["weights"][s], w_rule, rtol=1e-6, atol=1e-7), s
        if thr.cut in (lcf.CUT_FIXED_K, lcf.CUT_KNEE, lcf.CUT_MEDIAN, lcf.CUT_SLOPE):
            w_rule, k_rule, curv, _ = O.rule_weights(lam_g, oracle_thr(thr))
            assert d["k"][s] == k_rule, (s, d["k"][s], k_rule)
            assert np.allclose(d["weights"][s], w_rule, atol=1e-6)
            if k_rule != res["k"][s]:
                if thr.cut == lcf.CUT_MEDIAN:
                    tie = median_tie(lam_o, thr.beta_median, k_rule, res["k"][s])
                elif thr.cut == lcf.CUT_SLOPE:
                    tie = slope_tie(lam_o, thr.slope_thr, k_rule, res["k"][s])
                else:
                    tie = knee_tie(res["curv"][s], k_rule, res["k"][s])
                assert tie, ("non-tie k flip", s, k_rule, res["k"][s])
                forced = True
    if forced:
        ew = d["weights"].astype(np.float64)
        res = O.filter_packet(iq, gy, gx, O.Threshold(cut=O.CUT_EXPLICIT, explicit_w=ew, pd_mode=thr.pd_mode),
                              **geo)
    e_fro = rel_fro(io, res["iq_out"])
    emax, e99, e999, npx = pd_db_error(pd, res["pd"], mask)
    say(f"   rel_fro={e_fro:.3e} pd_db max={emax:.2e} p99={e99:.2e} p99.9={e999:.2e} n={npx} forced={forced} "
         f"sweeps={d['sweeps'].min()}..{d['sweeps'].max()} rank={d['rank'].min()}..{d['rank'].max()}")
    assert e_fro <= tol_fro
    assert emax <= tol_db
    return e_fro, emax


