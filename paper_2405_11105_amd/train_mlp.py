"""Train the learned eigencomponent-weight network on the GPU with the library's
own forward/backward/Adam kernels, and evaluate it against the rule it replaces.

Teachers. ``rule`` (default): the adaptive-threshold weights of the plain rule
itself, the curvature cut (Eq. 6, beta 1) with sigmoid weights (Eq. 9); the
network learns the rule's map from spectrum to weights and the library's gate
(LCF_OPT_MLP_GATE) keeps the rule wherever the network's prediction strays by
0.1 dB or more. ``search``: for every training packet the filter runs with the
curvature rule and sigmoid weights at each scaling factor beta of a grid; the
beta whose power Doppler image has the highest CNR against the generator's
vessel masks is kept, and its per-subset weights become the targets. This is
the per-packet exhaustive beta search of the Experimental Studies section,
which the Discussion notes is impractical in real time: the network has to
produce the searched weights from one subset's spectrum alone (a different
filter from the rule, so the gate rejects it; it is evaluated without one).

CNR = 10 log10((mean PD_vessel - mean PD_background) / std PD_background) with
the background = pixels farther than 3 rows from any vessel (Data processing
and evaluation section).

  python -m paper_2405_11105_amd.train_mlp --train 782 --holdout 32 --out mlp.ckpt
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

BETAS = (0.5, 0.7, 1.0, 1.4, 2.0, 2.8)


def _make(args):
    kind, seed = args
    import synth
    spec = synth.spec_learned(seed) if kind == "learned" else synth.spec_clinical(seed, seed_base=0)
    iq, mask = synth.make_packet(spec)
    return seed, iq, mask


def cnr_db(pd, mask):
    """CNR (dB) of a PD map (torch, GPU) against a vessel mask (torch bool)."""
    import torch
    bg = ~mask
    for d in range(1, 4):
        bg &= ~torch.roll(mask, d, 0) & ~torch.roll(mask, -d, 0)
    b = pd[mask].double().mean()
    g = pd[bg].double()
    num = (b - g.mean()).clamp_min(1e-30)
    return float(10.0 * torch.log10(num / g.std()))


def packet_runs(ctx, lcf, iq, mask_t, grid, prec, betas=BETAS):
    """Filter one packet at every beta; returns (eigvals [S][nt], weights per beta, cnr per beta)."""
    import torch
    out_w, cnrs, lam = [], [], None
    for beta in betas:
        thr = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID, beta_knee=beta)
        _, pd, dg = ctx.filter(iq, grid[0], grid[1], thr, precision=prec, iq_out=False, diag=True)
        if lam is None:
            lam = dg["eigvals"].clone()
        out_w.append(dg["weights"].clone())
        cnrs.append(cnr_db(pd, mask_t))
    return lam, out_w, cnrs


def generate(ctx, lcf, kind, seeds, grid, prec, workers, log=None, teacher="search"):
    """Teacher data: eigvals [N][128] (float64, GPU), targets [N][128] (float32, GPU), info."""
    import torch
    lams, tgts, info = [], [], []
    seeds = list(seeds)
    t0 = time.time()
    ctxmp = mp.get_context("spawn")   # workers run numpy only and never touch the GPU
    with ctxmp.Pool(workers) as pool:
        for n, (seed, iq_np, mask_np) in enumerate(pool.imap(_make, [(kind, s) for s in seeds], chunksize=1)):
            if log and n % 50 == 0:
                log(f"teacher packet {n}/{len(seeds)} ({time.time() - t0:.0f} s)")
            iq = torch.from_numpy(iq_np).cuda()
            mask_t = torch.from_numpy(mask_np).cuda()
            betas = (1.0,) if teacher == "rule" else BETAS
            lam, ws, cnrs = packet_runs(ctx, lcf, iq, mask_t, grid, prec, betas=betas)
            best = int(np.argmax(cnrs))
            lams.append(lam)
            tgts.append(ws[best])
            info.append({"seed": int(seed), "best_beta": betas[best], "cnr": cnrs})
    return torch.cat(lams), torch.cat(tgts), info


def train(ctx, lam, tgt, epochs, batch, lr, seed=0, log=None):
    import torch
    n = lam.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device=lam.device)
    hist = []
    steps_per_epoch = max(1, n // batch)
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(lam.device)
        lr_ep = lr * 0.5 * (1.0 + math.cos(math.pi * ep / epochs))
        acc = 0.0
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            ctx.mlp_train_step(lam[idx].contiguous(), tgt[idx].contiguous(), lr_ep, loss_out=loss)
            acc += loss.item() if s == steps_per_epoch - 1 else 0.0
        hist.append(acc)
        if log:
            log(f"epoch {ep} lr {lr_ep:.2e} loss {acc:.4e}")
    return hist


def _pd_dev(pd, ref, mask_t):
    """|10 log10(pd / ref)| over pixels with ref >= 2 x its median outside the
    vessels dilated by 2 rows (p99, max)."""
    import torch
    bg = ~mask_t
    for d in range(1, 3):
        bg &= ~torch.roll(mask_t, d, 0) & ~torch.roll(mask_t, -d, 0)
    floor = torch.median(ref[bg])
    sel = ref >= 2 * floor
    dev = (10 * torch.log10(pd[sel] / ref[sel])).abs().double()
    return float(torch.quantile(dev, 0.99)), float(dev.max())


def evaluate(ctx, lcf, kind, seeds, grid, prec, workers, log=None):
    """Held-out comparison of the plain rule (beta = 1), the searched-beta
    teacher, the network alone (no gate) and the network behind the gate (the
    context's LCF_OPT_MLP_GATE; rejected subsets keep the plain rule): CNR of
    each, the power Doppler deviation of the network from the rule and from
    the teacher, and the gate's fallback rate."""
    import torch
    rows = []
    ctxmp = mp.get_context("spawn")   # workers run numpy only and never touch the GPU
    with ctxmp.Pool(workers) as pool:
        for n, (seed, iq_np, mask_np) in enumerate(pool.imap(_make, [(kind, s) for s in seeds], chunksize=1)):
            if log and n % 8 == 0:
                log(f"held-out packet {n}")
            iq = torch.from_numpy(iq_np).cuda()
            mask_t = torch.from_numpy(mask_np).cuda()
            _, ws, cnrs = packet_runs(ctx, lcf, iq, mask_t, grid, prec)
            best = int(np.argmax(cnrs))
            thr_t = lcf.Threshold(cut=lcf.CUT_EXPLICIT)
            _, pd_t, _ = ctx.filter(iq, grid[0], grid[1], thr_t, precision=prec, iq_out=False, explicit_w=ws[best])
            thr_r = lcf.Threshold(cut=lcf.CUT_KNEE, shape=lcf.SHAPE_SIGMOID)
            _, pd_r, _ = ctx.filter(iq, grid[0], grid[1], thr_r, precision=prec, iq_out=False)
            thr_m = lcf.Threshold(cut=lcf.CUT_MLP, shape=lcf.SHAPE_SIGMOID)
            _, pd_g, dg = ctx.filter(iq, grid[0], grid[1], thr_m, precision=prec, iq_out=False, diag=True)
            fallback = float(((dg["flags"] & lcf.FLAG_MLP_FALLBACK) != 0).float().mean())
            gate = dg["mlp_gate"].double()
            gate_mdb = ctx.options[lcf.OPT_MLP_GATE]
            ctx.set_option(lcf.OPT_MLP_GATE, -1)
            try:
                _, pd_m, _ = ctx.filter(iq, grid[0], grid[1], thr_m, precision=prec, iq_out=False)
            finally:
                ctx.set_option(lcf.OPT_MLP_GATE, gate_mdb)
            torch.cuda.synchronize()
            r = {"seed": int(seed), "best_beta": BETAS[best], "cnr_rule": cnrs[BETAS.index(1.0)],
                 "cnr_teacher": cnrs[best], "cnr_mlp": cnr_db(pd_m, mask_t), "cnr_gated": cnr_db(pd_g, mask_t),
                 "fallback_rate": fallback, "gate_db_median": float(torch.median(gate))}
            for name, pd in (("mlp", pd_m), ("gated", pd_g)):
                for refn, ref in (("rule", pd_r), ("teacher", pd_t)):
                    p99, mx = _pd_dev(pd, ref, mask_t)
                    r[f"pd_db_{name}_vs_{refn}_p99"] = p99
                    r[f"pd_db_{name}_vs_{refn}_max"] = mx
            rows.append(r)
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--kind", default="learned", choices=["learned", "clinical"])
    ap.add_argument("--train", type=int, default=782, help="training packets")
    ap.add_argument("--holdout", type=int, default=32)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--precision", default="bf16x3", choices=["fp32", "bf16x3"])
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--out", default="mlp.ckpt")
    ap.add_argument("--report", default=None)
    ap.add_argument("--teacher", default="rule", choices=["rule", "search"])
    ap.add_argument("--eval-only", default=None, metavar="CKPT",
                    help="skip the teacher data and training; evaluate this checkpoint on the held-out packets")
    ap.add_argument("--gate-mdb", type=int, default=100, help="LCF_OPT_MLP_GATE for the evaluation")
    args = ap.parse_args(argv)
    import torch
    import paper_2405_11105_amd as lcf
    grid = (16, 16) if args.kind == "learned" else (8, 8)
    base_train, base_hold = (10000, 20000) if args.kind == "learned" else (5000, 6000)
    prec = lcf.PREC_BF16X3 if args.precision == "bf16x3" else lcf.PREC_FP32
    log = lambda m: print(m, flush=True)
    ctx = lcf.Context(0)
    ctx.set_option(lcf.OPT_MLP_GATE, args.gate_mdb)
    hist, info = [], []
    if args.eval_only:
        ctx.mlp_load(args.eval_only)
    else:
        t0 = time.time()
        lam, tgt, info = generate(ctx, lcf, args.kind, range(base_train, base_train + args.train), grid, prec,
                                  args.workers, log=log, teacher=args.teacher)
        log(f"teacher data: {lam.shape[0]} spectra from {args.train} packets in {time.time() - t0:.1f} s; "
            f"best beta histogram {np.unique([i['best_beta'] for i in info], return_counts=True)}")
        ctx.mlp_init(1)
        t1 = time.time()
        hist = train(ctx, lam, tgt, args.epochs, args.batch, args.lr, log=log)
        log(f"training: {time.time() - t1:.1f} s")
        ctx.mlp_save(args.out)
    rows = evaluate(ctx, lcf, args.kind, range(base_hold, base_hold + args.holdout), grid, prec, args.workers,
                    log=log)
    summ = {k: float(np.mean([r[k] for r in rows])) for k in rows[0] if k not in ("seed", "best_beta")}
    log("held-out mean: " + json.dumps(summ))
    if args.report:
        with open(args.report, "w") as f:
            json.dump({"summary": summ, "rows": rows, "loss": hist, "teacher": args.teacher,
                       "epochs": args.epochs, "train_info": info}, f)
    ctx.close()
    return summ


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()
