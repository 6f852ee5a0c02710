"""Image-quality study on synthetic recordings, the analogue of the paper's
Results: contrast ratio and contrast-to-noise ratio of the power Doppler image
(Experimental Studies: data processing and evaluation) as a function of each
thresholding method's scaling factor, for global, 2 x 2 and 3 x 3 processing
(recombined by Eq. 13 as written, and with its window compensation), over
packets sliding along a recording; the maximum over the factor is the
method's best achievable value (the exhaustive search of that section), and a
packet-size sweep (50, 70, 90 frames) with method 1.

  CR  = 10 log10(mean PD_blood / mean PD_background)
  CNR = 10 log10((mean PD_blood - mean PD_background) / std PD_background)

Blood ROI = the generator's vessel pixels; background ROI = pixels at the
vessels' depths (rows within 12 px of a vessel) that are more than 3 px from
every vessel. Every packet runs through the library on the GPU (sliding
packets: lcf_stream_push, the covariance carried between packets); the mean
and SD are over the packets of the recording. Times are device time per
packet with HIP events.

  python -m paper_2405_11105_amd.quality [--packets 16] [--json out.json]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import numpy as np

# scaling-factor grids per method (the Adaptive Thresholding Methods section)
METHODS = {
    "1 curvature (Eq. 6)": ("knee", [0.05, 0.1, 0.2, 0.3, 0.5, 0.7, 1.0, 1.4, 2.0]),
    "2 slope (Fig. 2c)": ("slope", [0.005, 0.01, 0.02, 0.05, 0.1, 0.2, 0.4, 1.1]),
    "3 median (Eq. 7)": ("median", [1.43, 2.0, 4.0, 8.0, 16.0, 32.0, 64.0]),
    "4 NCC (Eq. 8)": ("ncc", [None]),
    "5 NCC + sigmoid (Eq. 9)": ("ncc_sig", [0.5, 1.0, 2.0, 4.0, 8.0]),
    "6 eigenvalue power (Eq. 10)": ("power", [0.25, 0.5, 1.0, 1.5, 2.0, 3.0]),
}
# (gy, gx, sigma_frac, pd_mode): Eq. 13 as written, and with the window
# compensation (divided by sum_d alpha_d w_d^2) that removes the ripple the
# literal recombination leaves with sigma = spacing / 3
GRIDS = {"global": (1, 1, 0.0, 0), "2x2": (2, 2, 1.0 / 3.0, 0), "3x3": (3, 3, 1.0 / 3.0, 0),
         "2x2 compensated": (2, 2, 1.0 / 3.0, 2), "3x3 compensated": (3, 3, 1.0 / 3.0, 2)}


def threshold(lcf, kind, beta, pd_mode=0):
    T = lambda **kw: lcf.Threshold(pd_mode=pd_mode, **kw)
    if kind == "knee":
        return T(cut=lcf.CUT_KNEE, beta_knee=beta)
    if kind == "slope":
        return T(cut=lcf.CUT_SLOPE, slope_thr=beta)
    if kind == "median":
        return T(cut=lcf.CUT_MEDIAN, beta_median=beta)
    if kind == "ncc":
        return T(cut=lcf.CUT_NCC)
    if kind == "ncc_sig":
        return T(cut=lcf.CUT_NCC, shape=lcf.SHAPE_SIGMOID, beta_sigmoid=beta)
    if kind == "power":
        return T(cut=lcf.CUT_POWER, beta_power=beta)
    raise ValueError(kind)


def rois(mask):
    """Blood and background ROI masks (numpy bool [ny][nx])."""
    ny, nx = mask.shape
    near = np.zeros_like(mask)
    rows = np.where(mask.any(axis=1))[0]
    for r in rows:
        near[max(0, r - 12):min(ny, r + 13), :] = True
    far = ~mask
    for d in range(1, 4):
        far &= ~np.roll(mask, d, 0) & ~np.roll(mask, -d, 0)
    return mask, near & far


def cr_cnr(pd, blood, bg):
    b = pd[blood].double().mean()
    g = pd[bg].double()
    gm = g.mean()
    cr = 10.0 * math.log10(float(b / gm))
    num = float(b - gm)
    cnr = 10.0 * math.log10(num / float(g.std())) if num > 0 else float("-inf")
    return cr, cnr


def recording(ny, nx, nt, hop, packets, seed):
    """Phantom-like recording: 50 dB tissue with 0.5 px axial motion, four
    horizontal vessels of radius 2..6 px at 0.1..0.8 px/frame."""
    import synth
    tubes = ((ny // 5, 6, 0.8), (2 * ny // 5, 4, 0.4), (3 * ny // 5, 3, 0.2), (4 * ny // 5, 2, 0.1))
    spec = synth.PacketSpec(ny, nx, nt + hop * (packets - 1), 50.0, 0.5, tubes, seed=seed)
    return synth.make_packet(spec)


def recording_het(ny, nx, nt, hop, packets, seed):
    """Spatially uneven recording: the upper half holds slow, weaker tissue
    (0.1 px motion, 40 dB), the lower half fast, stronger tissue (1 px, 55 dB),
    two vessels in each; one global cut cannot suit both halves."""
    import synth
    h = ny // 2
    tot = nt + hop * (packets - 1)
    a = synth.PacketSpec(h, nx, tot, 40.0, 0.1, ((h // 3, 4, 0.5), (2 * h // 3, 2, 0.1)), seed=seed)
    b = synth.PacketSpec(ny - h, nx, tot, 55.0, 1.0, ((h // 3, 4, 0.5), (2 * h // 3, 2, 0.1)), seed=seed + 1)
    (ia, ma), (ib, mb) = synth.make_packet(a), synth.make_packet(b)
    return np.ascontiguousarray(np.concatenate([ia, ib], axis=1)), np.concatenate([ma, mb], axis=0)


def run_series(lcf, ctx, rec_t, nt, hop, packets, grid, thr, blood, bg, stream):
    """CR / CNR per packet and device ms per packet for one setting."""
    import torch
    gy, gx, sf, _ = grid
    ny, nx = rec_t.shape[1:]
    sm = lcf.Stream(ctx, ny, nx, nt, gy, gx, thr, precision=lcf.PREC_FP32, sigma_frac=sf)
    out = (torch.empty((nt, ny, nx), dtype=torch.complex64, device=rec_t.device),
           torch.empty((ny, nx), dtype=torch.float32, device=rec_t.device))
    crs, cnrs = [], []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = 0.0
    try:
        for p in range(packets):
            pk = rec_t[p * hop:p * hop + nt]
            e0.record(stream)
            sm.push(pk, hop, out=out)
            e1.record(stream)
            torch.cuda.synchronize()
            if p > 0:
                ms += e0.elapsed_time(e1)
            cr, cnr = cr_cnr(out[1], blood, bg)
            crs.append(cr)
            cnrs.append(cnr)
    finally:
        sm.close()
    if ctx.sync() != 0:
        raise RuntimeError("device-side condition flagged")
    return (float(np.mean(crs)), float(np.std(crs)), float(np.mean(cnrs)), float(np.std(cnrs)),
            ms / max(1, packets - 1))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--ny", type=int, default=196)
    ap.add_argument("--nx", type=int, default=180)
    ap.add_argument("--nt", type=int, default=50)
    ap.add_argument("--hop", type=int, default=5)
    ap.add_argument("--packets", type=int, default=16)
    ap.add_argument("--seed", type=int, default=4000)
    ap.add_argument("--json", default=None)
    args = ap.parse_args(argv)
    import torch
    import paper_2405_11105_amd as lcf
    ctx = lcf.Context(0)
    stream = torch.cuda.current_stream()
    res = {"methods": {}, "packet_size": {}, "uneven_tissue": {}}
    rec, mask = recording(args.ny, args.nx, 90, args.hop, args.packets, args.seed)
    blood, bg = (torch.from_numpy(m).cuda() for m in rois(mask))
    rec_t = torch.from_numpy(rec).cuda()
    for mname, (kind, betas) in METHODS.items():
        for gname, grid in GRIDS.items():
            rows = []
            for beta in betas:
                thr = threshold(lcf, kind, beta, grid[3])
                rows.append((beta,) + run_series(lcf, ctx, rec_t[:args.nt + args.hop * (args.packets - 1)],
                                                 args.nt, args.hop, args.packets, grid, thr, blood, bg, stream))
            res["methods"].setdefault(mname, {})[gname] = rows
            print(f"{mname:30s} {gname:16s} best CR {max(r[1] for r in rows):6.2f} dB  best CNR "
                  f"{max(r[3] for r in rows):6.2f} dB  {np.mean([r[5] for r in rows]):.3f} ms/packet", flush=True)
    for nt in (50, 70, 90):
        for gname, grid in GRIDS.items():
            rows = []
            for beta in METHODS["1 curvature (Eq. 6)"][1]:
                thr = threshold(lcf, "knee", beta, grid[3])
                rows.append((beta,) + run_series(lcf, ctx, rec_t[:nt + args.hop * (args.packets - 1)], nt,
                                                 args.hop, args.packets, grid, thr, blood, bg, stream))
            res["packet_size"].setdefault(str(nt), {})[gname] = rows
            print(f"method 1 Nt={nt} {gname:16s} best CR {max(r[1] for r in rows):6.2f} dB  best CNR "
                  f"{max(r[3] for r in rows):6.2f} dB  {np.mean([r[5] for r in rows]):.3f} ms/packet", flush=True)
    # spatially uneven tissue: where local processing should pay (method 1)
    rec2, mask2 = recording_het(args.ny, args.nx, args.nt, args.hop, args.packets, args.seed + 7)
    blood2, bg2 = (torch.from_numpy(m).cuda() for m in rois(mask2))
    rec2_t = torch.from_numpy(rec2).cuda()
    for gname, grid in GRIDS.items():
        rows = []
        for beta in METHODS["1 curvature (Eq. 6)"][1]:
            thr = threshold(lcf, "knee", beta, grid[3])
            rows.append((beta,) + run_series(lcf, ctx, rec2_t, args.nt, args.hop, args.packets, grid, thr, blood2,
                                             bg2, stream))
        res["uneven_tissue"][gname] = rows
        print(f"uneven tissue, method 1 {gname:16s} best CR {max(r[1] for r in rows):6.2f} dB  best CNR "
              f"{max(r[3] for r in rows):6.2f} dB", flush=True)
    ctx.close()
    # summary table (markdown)
    lines = ["| method | processing | best CR (dB) at factor | best CNR (dB) at factor | ms / packet |",
             "|---|---|---|---|---|"]
    for mname, by in res["methods"].items():
        for gname, rows in by.items():
            icr = int(np.argmax([r[1] for r in rows]))
            icn = int(np.argmax([r[3] for r in rows]))
            f = lambda b: "-" if b is None else f"{b:g}"
            lines.append(f"| {mname} | {gname} | {rows[icr][1]:.2f} +- {rows[icr][2]:.2f} at {f(rows[icr][0])} | "
                         f"{rows[icn][3]:.2f} +- {rows[icn][4]:.2f} at {f(rows[icn][0])} | "
                         f"{np.mean([r[5] for r in rows]):.3f} |")
    lines += ["", "| packet size (method 1) | processing | best CR (dB) | best CNR (dB) | ms / packet |",
              "|---|---|---|---|---|"]
    for nt, by in res["packet_size"].items():
        for gname, rows in by.items():
            lines.append(f"| {nt} | {gname} | {max(r[1] for r in rows):.2f} | {max(r[3] for r in rows):.2f} | "
                         f"{np.mean([r[5] for r in rows]):.3f} |")
    lines += ["", "| uneven tissue (method 1) | best CR (dB) | best CNR (dB) |", "|---|---|---|"]
    for gname, rows in res["uneven_tissue"].items():
        lines.append(f"| {gname} | {max(r[1] for r in rows):.2f} | {max(r[3] for r in rows):.2f} |")
    table = "\n".join(lines)
    print(table)
    if args.json:
        with open(args.json, "w") as f:
            json.dump({"args": vars(args), "results": res, "table": table}, f)
    return res


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()
