"""Train the learned unrolled FISTA on synthetic scenes of the paper-scale geometry.

python -m paper_2509_13592_amd.train_lista [--train-scenes N] [--steps S] [--out weights.json]

Scenes: the fixed 16x16-URA mask with 64 elements, L1 = L2 = 256, K ~ U{1..8}
targets, SNR ~ U[10, 30] dB (training split 0).  Labels: plain FISTA with
`--label-iters` iterations from zero (batched solver on the GPU).  The default
target is 200 iterations: 16 layers can learn to reproduce it (relative error
~0.27), while 2000-iteration labels are out of their reach (~0.9) and only pull
the network towards near-zero outputs.  The network,
its backward and Adam all run in the HIP library; this script only drives them.
The result is a JSON file with the 16 x 52 parameters and the training record.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "weights", "lista16_paper256.json")


def make_split(B, plan, split, start, count, mask, chunk=2048):
    import torch
    from . import scenes as S
    ys = np.stack([S.learned_scene(split, start + i, mask).y for i in range(count)])
    ys = B.to_device(ys)
    taus = np.array([np.float32(0.1 * plan.adjoint_maxabs(ys[i])) for i in range(count)], dtype=np.float32)
    return ys, taus


def labels_for(B, plan, ys, taus, iters, chunk=2048):
    import torch
    n = ys.shape[0]
    out = torch.empty((n, plan.L2, plan.L1), dtype=torch.complex64, device=ys.device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        batch = B.Batch([plan] * (e - s))
        batch.fista([ys[i] for i in range(s, e)], taus[s:e].tolist(), iters, outs=[out[i] for i in range(s, e)])
        batch.close()
    return out


def train(args):
    import torch
    from . import bccb as B
    from . import scenes as S
    torch.cuda.set_device(0)
    mask = S.learned_fixed_mask()
    plan = B.Plan(mask, 256, 256)
    t0 = time.time()
    ys, taus = make_split(B, plan, 0, 0, args.train_scenes, mask)
    labels = labels_for(B, plan, ys, taus, args.label_iters)
    torch.cuda.synchronize()
    t_label = time.time() - t0
    print(f"labels: {args.train_scenes} scenes x {args.label_iters} FISTA iterations in {t_label:.1f} s", flush=True)
    vys, vtaus = make_split(B, plan, 1, 0, args.val_scenes, mask)
    vlab = labels_for(B, plan, vys, vtaus, args.label_iters)

    K = args.layers
    net = B.Lista(plan, layers=K, max_batch=max(args.batch, args.val_scenes), train=True)
    params = B.lista_init_params(K)
    opt = B.Adam(params, lr=args.lr, lr_scale=B.lista_lr_scale(K, args.delta_lr_scale))
    rng = np.random.default_rng(args.seed)

    def val_loss():
        net.forward(params, vys, vtaus)
        _, l = net.backward(params, vlab)
        return l

    curve = [(0, val_loss())]
    print(f"step 0 val loss {curve[-1][1]:.5f}", flush=True)
    t1 = time.time()
    step = 0
    while step < args.steps:
        perm = rng.permutation(args.train_scenes)
        for s in range(0, args.train_scenes - args.batch + 1, args.batch):
            idx = torch.from_numpy(np.sort(perm[s:s + args.batch])).to(ys.device)
            yb = ys.index_select(0, idx).contiguous()
            lb = labels.index_select(0, idx).contiguous()
            tb = taus[np.sort(perm[s:s + args.batch])]
            net.forward(params, yb, tb)
            g, loss = net.backward(params, lb)
            if not np.isfinite(loss):
                raise RuntimeError(f"non-finite training loss at step {step}")
            opt.step(g)
            step += 1
            if step % args.log_every == 0 or step == args.steps:
                curve.append((step, val_loss()))
                print(f"step {step} train loss {loss:.5f} val loss {curve[-1][1]:.5f}", flush=True)
            if step >= args.steps:
                break
    torch.cuda.synchronize()
    t_train = time.time() - t1
    rec = {
        "layers": K,
        "per_layer": ["s", "theta"] + [f"re_delta[{a}][{b}]" for a in range(5) for b in range(5)]
                     + [f"im_delta[{a}][{b}]" for a in range(5) for b in range(5)],
        "params": params.cpu().numpy().astype(float).tolist(),
        "geometry": {"M1": 16, "M2": 16, "M": int(mask.sum()), "L1": 256, "L2": 256,
                     "mask_seed": [5, 0, 0]},
        "train_scenes": args.train_scenes, "label_iters": args.label_iters, "batch": args.batch,
        "steps": args.steps, "lr": args.lr, "delta_lr_scale": args.delta_lr_scale, "val_scenes": args.val_scenes,
        "val_loss_curve": curve, "label_seconds": round(t_label, 2), "train_seconds": round(t_train, 2),
    }
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {args.out}: val loss {curve[0][1]:.5f} -> {curve[-1][1]:.5f} in {t_train:.1f} s", flush=True)
    net.close()
    return rec


def load_params(path=DEFAULT_OUT, device="cuda"):
    import torch
    with open(path) as f:
        rec = json.load(f)
    return torch.tensor(np.asarray(rec["params"], dtype=np.float32), device=device), rec


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-scenes", type=int, default=8192)
    ap.add_argument("--val-scenes", type=int, default=256)
    ap.add_argument("--label-iters", type=int, default=200)
    ap.add_argument("--layers", type=int, default=16)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--lr", type=float, default=0.005)
    ap.add_argument("--delta-lr-scale", type=float, default=0.01)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--log-every", type=int, default=50)
    ap.add_argument("--out", default=DEFAULT_OUT)
    args = ap.parse_args(argv)
    train(args)


if __name__ == "__main__":
    sys.exit(main())
