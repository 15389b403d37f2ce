"""Train the warm-start network on solutions of the EMD iteration itself.

    python -m paper_1805_09453_amd.warmstart_train --pairs 20000 --epochs 30 --batch 32 --native 128 \
        --out paper_1805_09453_amd/weights/ws_unet.f32 --summary paper_1805_09453_amd/weights/ws_unet.json

Steps (everything numerical runs in libgprox on the GPU; this module only
moves tensors and loops):
  1. seeded 512x512 density pairs, each a mixture of K ~ U{4..16} isotropic
     Gaussians (synth.emd_mixture_pair, seed = config_seed(4, i));
  2. target potentials phi*: gp_batch_solve (the plain zero-start iteration of
     section 3.2) to --target-tol, returning the scaled certificate potential;
  3. the network runs at --native (a divisor of 512): densities and targets are
     block-averaged to it with ws_downsample (a coarser native size widens the
     network's receptive field relative to the domain; the potential is smooth);
     training with ws_grads / ws_adam (mean squared gradient error, Adam with a
     cosine learning-rate decay), a held-out slice monitored for the loss;
  4. evaluation on held-out 512^2 pairs: plain emd_solve vs ws_emd_solve
     (block mean to the native size, prediction, bilinear interpolation,
     certificate check and any fallback included) to --eval-tol;
  5. the FP32 parameter blob is written to --out (raw little-endian floats).
"""
import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

N_NATIVE = 512
EVAL_OFFSET = 900_000  # held-out seeds: config_seed(4, EVAL_OFFSET + j)


def pair(i: int, n: int = N_NATIVE):
    """Pair i of the training distribution: K ~ U{4..16} Gaussians per density."""
    seed = synth.config_seed(4, i)
    k = int(np.random.default_rng(seed).integers(4, 17))
    r0, r1 = synth.emd_mixture_pair(n, seed, k=k)
    return r0.astype(np.float32), r1.astype(np.float32)


def _pair_n(args):
    return pair(*args)


def make_pairs(ids, n=N_NATIVE, workers=16):
    with ProcessPoolExecutor(workers) as ex:
        out = list(ex.map(_pair_n, [(i, n) for i in ids], chunksize=8))
    return np.stack([a for a, _ in out]), np.stack([b for _, b in out])


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def targets(ctx, R0, R1, tol, max_iter, chunk=256):
    """phi* for every pair via gp_batch_solve; returns (phi*, iteration counts)."""
    import torch

    from . import Options
    from ._lib import GP_KIND_EMD
    N, n = R0.shape[0], R0.shape[1]
    PHI = torch.empty_like(R0)
    iters = []
    for s in range(0, N, chunk):
        probs = []
        for i in range(s, min(N, s + chunk)):
            probs.append({"kind": GP_KIND_EMD, "rho0": R0[i], "rho1": R1[i], "h": 1.0 / n, "tau": 0.3,
                          "phi": PHI[i]})
        t0 = time.time()
        _, reps, _ = ctx.batch_solve(probs, Options(tau=0.3, tol=tol, max_iter=max_iter, check_every=20))
        torch.cuda.synchronize()
        iters += [r["iters"] for r in reps]
        log(f"targets {s + len(probs)}/{N}: {time.time() - t0:.1f}s, median iters "
            f"{int(np.median([r['iters'] for r in reps]))}, converged {sum(r['converged'] for r in reps)}")
    return PHI, iters


def symmetry(a, c, t, code):
    """One of the 16 symmetries of a pair on the square: the 8 rotations and
    reflections of the grid (the potential moves with the densities) and the
    exchange of the two densities (the potential changes sign).  Index
    permutations and a sign only."""
    import torch
    if code & 1:
        a, c, t = (torch.flip(x, dims=(-1,)) for x in (a, c, t))
    if code & 2:
        a, c, t = (torch.flip(x, dims=(-2,)) for x in (a, c, t))
    if code & 4:
        a, c, t = (x.transpose(-1, -2) for x in (a, c, t))
    if code & 8:
        a, c, t = c, a, -t
    return a.contiguous(), c.contiguous(), t.contiguous()


def train(ws, R0, R1, PHI, epochs, batch, lr, val=32, seed=0, augment=True):
    import torch
    N, n = R0.shape[0], R0.shape[1]
    ntr = N - val
    steps = epochs * (ntr // batch)
    rng = np.random.default_rng(seed)
    hist, t0, step = [], time.time(), 0
    for ep in range(epochs):
        perm = rng.permutation(ntr)
        tr = []
        for b in range(ntr // batch):
            idx = torch.tensor(perm[b * batch:(b + 1) * batch], device=R0.device)
            a, c, t = R0.index_select(0, idx), R1.index_select(0, idx), PHI.index_select(0, idx)
            if augment:
                a, c, t = symmetry(a, c, t, int(rng.integers(16)))
            tr.append(ws.grads(a, c, t, 1.0 / n))
            cur = lr * 0.5 * (1 + math.cos(math.pi * step / steps))
            ws.adam(cur)
            step += 1
        vl = []
        for b in range(0, val, batch):
            sl = slice(ntr + b, ntr + min(val, b + batch))
            vl.append(ws.grads(R0[sl].contiguous(), R1[sl].contiguous(), PHI[sl].contiguous(), 1.0 / n))
        hist.append({"epoch": ep, "train_loss": float(np.mean(tr)), "val_loss": float(np.mean(vl)),
                     "seconds": time.time() - t0})
        log(f"epoch {ep}: train {hist[-1]['train_loss']:.4e} val {hist[-1]['val_loss']:.4e} "
            f"({hist[-1]['seconds']:.0f}s, {step} steps)")
    return hist


def evaluate(ctx, ws, E0, E1, tol, max_iter, n=N_NATIVE):
    import torch

    from . import Options
    count = E0.shape[0]
    R0, R1 = torch.tensor(E0, device="cuda"), torch.tensor(E1, device="cuda")
    opts = Options(tau=0.3, tol=tol, max_iter=max_iter, check_every=20)
    rows = []
    for j in range(count):
        torch.cuda.synchronize()
        t0 = time.time()
        _, _, rp = ctx.emd_solve(R0[j], R1[j], 1.0 / n, opts, want_phi=False)
        torch.cuda.synchronize()
        tp = time.time() - t0
        t0 = time.time()
        _, _, rw, wr = ws.emd_solve(R0[j], R1[j], 1.0 / n, opts)
        torch.cuda.synchronize()
        tw = time.time() - t0
        iters_w = rw["iters"] + (wr["warm_iters"] if wr["fallback"] else 0)
        rows.append({"plain_iters": rp["iters"], "plain_s": tp, "warm_iters": iters_w, "warm_s": tw,
                     "fallback": wr["fallback"], "d0": wr["d0"], "plain_dual": rp["dual"], "warm_primal": rw["primal"],
                     "converged": bool(rp["converged"] and rw["converged"])})
        log(f"eval {j}: plain {rp['iters']} it {tp:.3f}s | warm {iters_w} it {tw:.3f}s fallback {wr['fallback']}")
    sp = sum(r["plain_s"] for r in rows)
    sw = sum(r["warm_s"] for r in rows)
    return {"pairs": count, "tol": tol, "rows": rows,
            "plain_iters_total": sum(r["plain_iters"] for r in rows),
            "warm_iters_total": sum(r["warm_iters"] for r in rows),
            "plain_seconds_total": sp, "warm_seconds_total": sw, "speedup": sp / sw if sw > 0 else None,
            "fallbacks": sum(r["fallback"] for r in rows)}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--target-tol", type=float, default=1e-4)
    ap.add_argument("--target-max-iter", type=int, default=8000)
    ap.add_argument("--eval-pairs", type=int, default=16)
    ap.add_argument("--eval-tol", type=float, default=1e-5)
    ap.add_argument("--eval-max-iter", type=int, default=40000)
    ap.add_argument("--init-seed", type=int, default=1)
    ap.add_argument("--native", type=int, default=128, help="network resolution (divides 512)")
    ap.add_argument("--no-augment", action="store_true", help="train without the 16 grid/exchange symmetries")
    ap.add_argument("--out", required=True)
    ap.add_argument("--summary")
    a = ap.parse_args(argv)
    import torch

    from . import Context, WarmStart
    n = N_NATIVE
    t_all = time.time()
    log(f"generating {a.pairs} + {a.eval_pairs} pairs at {n}x{n}")
    # all host-side generation happens before the GPU is first touched (worker processes fork)
    E0, E1 = make_pairs([EVAL_OFFSET + j for j in range(a.eval_pairs)], n) if a.eval_pairs else (None, None)
    R0, R1 = make_pairs(range(a.pairs), n)
    R0, R1 = torch.tensor(R0, device="cuda"), torch.tensor(R1, device="cuda")
    ctx = Context(n, n)
    log("solving targets")
    PHI, titers = targets(ctx, R0, R1, a.target_tol, a.target_max_iter)
    nn = a.native
    f = n // nn
    if f > 1:
        from . import ws_downsample
        log(f"block-averaging inputs and targets {n} -> {nn}")
        down = lambda X: torch.stack([ws_downsample(ctx, X[i], f) for i in range(X.shape[0])])
        R0, R1, PHI = down(R0), down(R1), down(PHI)
        torch.cuda.synchronize()
    ws = WarmStart(ctx, a.batch, nn, nn)
    # He-normal initial weights (fan-in), zero biases, seeded; the 1x1 head starts at zero
    # so the first prediction is phi = 0 (loss = mean |grad phi*|^2) instead of noise
    rng = np.random.default_rng(a.init_seed)
    blob = np.zeros(ws.n_params, dtype=np.float32)
    o = 0
    for kind, cin, cout in LAYERS:
        nw = {"conv3": 9 * cin * cout, "tconv2": 4 * cin * cout, "conv1": cin * cout}[kind]
        fan = {"conv3": 9 * cin, "tconv2": cin, "conv1": cin}[kind]
        if kind != "conv1":
            blob[o:o + nw] = rng.standard_normal(nw) * math.sqrt(2.0 / fan)
        o += nw + cout
    assert o == ws.n_params
    ws.set_params(torch.tensor(blob, device="cuda"))
    log("training")
    hist = train(ws, R0, R1, PHI, a.epochs, a.batch, a.lr, augment=not a.no_augment)
    params = ws.get_params().cpu().numpy()
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    params.astype("<f4").tofile(a.out)
    log(f"weights written to {a.out}")
    del R0, R1, PHI
    torch.cuda.empty_cache()
    ev = evaluate(ctx, ws, E0, E1, a.eval_tol, a.eval_max_iter) if a.eval_pairs else None
    summary = {"pairs": a.pairs, "native": nn, "solve_grid": n, "epochs": a.epochs, "batch": a.batch, "lr": a.lr,
               "augment": not a.no_augment,
               "target_tol": a.target_tol, "target_iters_median": int(np.median(titers)),
               "history": hist, "eval": ev, "seconds": time.time() - t_all}
    if a.summary:
        with open(a.summary, "w") as fh:
            json.dump(summary, fh, indent=1)
    if ev:
        log(f"held-out: plain {ev['plain_iters_total']} it / {ev['plain_seconds_total']:.2f}s, warm "
            f"{ev['warm_iters_total']} it / {ev['warm_seconds_total']:.2f}s, fallbacks {ev['fallbacks']}")
    ws.close()
    ctx.close()


# (kind, cin, cout) in parameter-blob order (the layout documented in include/gprox.h)
LAYERS = [("conv3", 2, 32), ("conv3", 32, 32), ("conv3", 32, 64), ("conv3", 64, 64), ("conv3", 64, 128),
          ("conv3", 128, 128), ("conv3", 128, 256), ("conv3", 256, 256), ("tconv2", 256, 128), ("conv3", 256, 128),
          ("conv3", 128, 128), ("tconv2", 128, 64), ("conv3", 128, 64), ("conv3", 64, 64), ("tconv2", 64, 32),
          ("conv3", 64, 32), ("conv3", 32, 32), ("conv1", 32, 1)]

if __name__ == "__main__":
    main()
