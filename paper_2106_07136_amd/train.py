"""Training driver of the proposal network.

Generated 640x480 pairs -> plain BDIS on the GPU (the disparities the network
learns from) -> targets on the 1/16 grid (block mean of the estimated
disparities, in 1/16-level pixels) and network inputs (bdis_net_input) ->
forward, loss, backward and Adam through the bdisnet kernels.  Pair
generation runs in a pool of worker processes while the GPU works.

    python -m paper_2106_07136_amd.train --sizes 640x480:64:20000:10000 --channels 32 \
        --out proposal_c{C}.npz
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import synth


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _gen(args):
    W, H, d, s = args
    p = synth.make_pair(W, H, d, s)
    return p.left, p.right


def targets_from_disparity(d, factor=16, min_frac=0.5):
    """d: (N, H, W) float tensor, NaN = not estimated.  Returns (target,
    valid) on the grid of the 1/16 level: mean of the estimated disparities
    of each factor x factor block divided by factor, valid where at least
    min_frac of the block is estimated."""
    import torch
    N, H, W = d.shape
    h4, w4 = H, W
    for _ in range(int(round(math.log2(factor)))):
        h4, w4 = (h4 + 1) // 2, (w4 + 1) // 2
    pad = torch.full((N, h4 * factor, w4 * factor), float("nan"), device=d.device)
    pad[:, :H, :W] = d
    b = pad.view(N, h4, factor, w4, factor)
    fin = torch.isfinite(b)
    cnt = fin.sum(dim=(2, 4)).float()
    s = torch.where(fin, b, torch.zeros_like(b)).sum(dim=(2, 4))
    tgt = torch.where(cnt > 0, s / cnt.clamp(min=1) / factor, torch.zeros_like(s))
    valid = cnt >= min_frac * factor * factor
    return tgt.float().contiguous(), valid.to(torch.uint8).contiguous()


def build_dataset(sizes, workers, chunk):
    """sizes: list of (W, H, d_max, n, seed0).  Generates the pairs of every
    size and returns one (X, T, V) triple of GPU tensors per size.  With
    workers > 1 the pairs come from a forked pool, which must be started
    before this process touches the GPU; workers <= 1 generates in-process."""
    import multiprocessing as mp
    spec = [(W, H, d, s0 + i) for (W, H, d, n, s0) in sizes for i in range(n)]
    pool = None
    if workers > 1:
        pool = mp.get_context("fork").Pool(workers)
        it = pool.imap(_gen, spec, chunksize=4)
    else:
        it = map(_gen, spec)
    import torch

    from . import bdis
    dev = torch.device("cuda:0")
    t0 = time.time()
    data = []
    for (W, H, d, n, s0) in sizes:
        h = bdis.Bdis(bdis.Params(levels=0, iters=12, max_disparity=d))
        X = T = V = None
        done = 0
        while done < n:
            b = min(chunk, n - done)
            pairs = [next(it) for _ in range(b)]
            L = [torch.from_numpy(l).to(dev) for l, _ in pairs]
            R = [torch.from_numpy(r).to(dev) for _, r in pairs]
            outs = h.compute_batch(L, R)
            x = h.net_input(L, R)
            tgt, val = targets_from_disparity(torch.stack(outs))
            if X is None:
                X = torch.empty((n,) + tuple(x.shape[1:]), dtype=torch.bfloat16, device=dev)
                T = torch.empty((n,) + tuple(tgt.shape[1:]), dtype=torch.float32, device=dev)
                V = torch.empty((n,) + tuple(val.shape[1:]), dtype=torch.uint8, device=dev)
            X[done:done + b] = x
            T[done:done + b] = tgt
            V[done:done + b] = val
            done += b
            log(f"train: data {W}x{H} {done}/{n} pairs ({time.time() - t0:.0f} s)")
        h.close()
        data.append((X, T, V))
    if pool is not None:
        pool.close()
        pool.join()
    return data


def train(data, channels=32, epochs=6, batch=64, lr=2e-3, seed=0, conf_tol=1.0, log_every=500,
          resume=None, stop_after=None, state_out=None):
    """data: list of (X, T, V) per image size; every step takes one batch of
    one size, the sizes interleaved in proportion to their counts.

    Resumable: `stop_after` ends the run after that many steps (counted from
    the start); `state_out`, a dict, receives the state to resume from (the
    network checkpoint with its Adam moments and step, the epoch, the
    position in the epoch and the data-order generator's state at the start
    of that epoch); `resume` takes such a state and continues the run as if
    it had not stopped, bit for bit."""
    import torch

    from . import net
    pn = net.ProposalNet(channels)
    pn.set_params(net.init_params(channels, seed))
    g = torch.Generator(device="cpu").manual_seed(seed)
    per_epoch = [(k, j) for k, (X, _, _) in enumerate(data) for j in range(X.shape[0] // batch)]
    total = epochs * len(per_epoch)
    loss_buf = torch.empty((), dtype=torch.float32, device=data[0][0].device)
    step, ep0, pos0, hist = 0, 0, 0, []
    if resume is not None:
        pn.load_checkpoint(resume["net"])
        step, ep0, pos0 = int(resume["step"]), int(resume["epoch"]), int(resume["pos"])
        hist = [tuple(h) for h in resume["hist"]]
        g.set_state(torch.from_numpy(np.asarray(resume["rng"], np.uint8).copy()))
        assert pn.step == step, "checkpoint step does not match the network's"
    t0 = time.time()

    def snapshot(ep, pos, rng):
        if state_out is not None:
            state_out.update(net=pn.save_checkpoint(), step=step, epoch=ep, pos=pos, rng=rng, hist=list(hist))

    for ep in range(ep0, epochs):
        rng_start = g.get_state().numpy().copy()
        perms = [torch.randperm(X.shape[0], generator=g).to(X.device) for (X, _, _) in data]
        order = torch.randperm(len(per_epoch), generator=g).tolist()
        for pos in range(pos0 if ep == ep0 else 0, len(order)):
            if stop_after is not None and step >= stop_after:
                snapshot(ep, pos, rng_start)
                return pn, hist
            k, j = per_epoch[order[pos]]
            X, T, V = data[k]
            idx = perms[k][j * batch:(j + 1) * batch]
            step += 1
            lr_t = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * (step - 1) / total)))
            pn.forward(X[idx].contiguous())
            pn.loss(T[idx].contiguous(), V[idx].contiguous(), delta=1.0, conf_tol=conf_tol, conf_weight=0.1,
                    out=loss_buf)
            pn.backward()
            pn.adam_step(lr_t, step)
            if step % log_every == 0 or step == total:
                lv = float(loss_buf.item())
                hist.append((step, lv))
                log(f"train: epoch {ep} step {step}/{total} loss {lv:.4f} lr {lr_t:.2e} ({time.time() - t0:.1f} s)")
    snapshot(epochs, 0, g.get_state().numpy().copy())
    return pn, hist


def save_state(path, state):
    """A resumable training state (train's state_out) as an .npz of plain
    arrays (no pickled objects)."""
    np.savez(path, net=np.frombuffer(state["net"], np.uint8), step=np.int64(state["step"]),
             epoch=np.int64(state["epoch"]), pos=np.int64(state["pos"]), rng=np.asarray(state["rng"], np.uint8),
             hist=np.array(json.dumps(state["hist"])))


def load_state(path):
    z = np.load(path, allow_pickle=False)
    return {"net": z["net"].tobytes(), "step": int(z["step"]), "epoch": int(z["epoch"]), "pos": int(z["pos"]),
            "rng": z["rng"], "hist": json.loads(str(z["hist"]))}


def save(path, pn, meta):
    np.savez(path, params=pn.get_params(), channels=np.int32(pn.channels),
             meta=np.array(json.dumps(meta)))


def load(path):
    """Returns (flat FP32 parameters, channels, meta dict); executes nothing
    from the file."""
    z = np.load(path, allow_pickle=False)
    return z["params"].astype(np.float32), int(z["channels"]), json.loads(str(z["meta"]))


def parse_sizes(text):
    """'640x480:64:20000:10000,1920x1080:192:2000:30000' -> [(W, H, d_max, n, seed0)]"""
    out = []
    for item in text.split(","):
        wh, d, n, s0 = item.split(":")
        W, H = wh.split("x")
        out.append((int(W), int(H), float(d), int(n), int(s0)))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="640x480:64:20000:10000",
                    help="comma list of WxH:max_disparity:pairs:first_seed")
    ap.add_argument("--channels", default="32", help="comma list: one network per width, same data")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--conf-tol", type=float, default=1.0)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--chunk", type=int, default=256)
    ap.add_argument("--out", required=True, help="output path; {C} is replaced by the width")
    ap.add_argument("--state", default=None,
                    help="resumable training state path ({C} replaced); resumed from when it exists, "
                         "written when the run stops")
    ap.add_argument("--stop-after", type=int, default=None, help="stop after this many steps (then resume)")
    a = ap.parse_args()
    sizes = parse_sizes(a.sizes)
    data = build_dataset(sizes, a.workers, a.chunk)
    for C in [int(c) for c in a.channels.split(",")]:
        spath = a.state.replace("{C}", str(C)) if a.state else None
        resume = load_state(spath) if spath and os.path.exists(spath) else None
        st = {}
        pn, hist = train(data, C, a.epochs, a.batch, a.lr, conf_tol=a.conf_tol, resume=resume,
                         stop_after=a.stop_after, state_out=st)
        if spath:
            save_state(spath, st)
            log(f"train: state saved to {spath} at step {st['step']}")
        if a.stop_after is not None and st["epoch"] < a.epochs:
            continue
        meta = {"sizes": sizes, "epochs": a.epochs, "batch": a.batch, "lr": a.lr, "conf_tol": a.conf_tol,
                "loss_history": hist}
        path = a.out.replace("{C}", str(C))
        save(path, pn, meta)
        log(f"train: saved {path}")


if __name__ == "__main__":
    main()
