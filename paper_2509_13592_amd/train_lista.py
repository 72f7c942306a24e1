"""Train the learned unrolled FISTA on synthetic scenes of the paper-scale geometry.

python -m paper_2509_13592_amd.train_lista [--spec] [--train-scenes N] [--steps S] [--out weights.json]

The packaged weights were made with --spec.

Scenes: the fixed 16x16-URA mask with 64 elements, L1 = L2 = 256, K ~ U{1..8}
targets, SNR ~ U[10, 30] dB (training split 0).  Labels: plain FISTA with
`--label-iters` iterations from zero (batched solver on the GPU).  The default
target is 200 iterations on 8192 scenes: 16 layers can learn to reproduce it (relative
error ~0.27).  --spec trains on the stated set instead: 2^20 scenes labelled by
2000-iteration FISTA, the labels kept sparse on the host.  The network,
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


class SparseLabels:
    """Labels kept sparse on the host: per scene the grid indices (int32) and values (complex64)
    of its nonzeros, concatenated, with offsets.  2^20 dense 256 x 256 labels would take 550 GB."""

    def __init__(self):
        self.idx, self.val, self.counts = [], [], []

    def add_dense_chunk(self, grids):
        import torch
        n = grids.shape[0]
        flat = grids.reshape(n, -1)
        nz = (flat.real != 0) | (flat.imag != 0)
        counts = nz.sum(dim=1).cpu().numpy()
        rows, cols = torch.nonzero(nz, as_tuple=True)
        self.idx.append(cols.to(torch.int32).cpu().numpy())
        self.val.append(flat[rows, cols].cpu().numpy().astype(np.complex64))
        self.counts.append(counts.astype(np.int64))

    def finish(self):
        self.idx = np.concatenate(self.idx)
        self.val = np.concatenate(self.val)
        self.counts = np.concatenate(self.counts)
        self.off = np.concatenate([[0], np.cumsum(self.counts)])

    def dense(self, scenes, L, device):
        """Dense complex64 [len(scenes)][L] labels of the given scene indices, on the device."""
        import torch
        out = torch.zeros((len(scenes), L), dtype=torch.complex64, device=device)
        parts_r, parts_i, parts_v = [], [], []
        for r, s in enumerate(scenes):
            a, b = self.off[s], self.off[s + 1]
            parts_r.append(np.full(b - a, r, dtype=np.int64))
            parts_i.append(self.idx[a:b].astype(np.int64))
            parts_v.append(self.val[a:b])
        rr = torch.from_numpy(np.concatenate(parts_r)).to(device)
        ii = torch.from_numpy(np.concatenate(parts_i)).to(device)
        vv = torch.from_numpy(np.concatenate(parts_v)).to(device)
        out[rr, ii] = vv
        return out


def spec_data(B, plan, mask, n, label_iters, chunk=4096):
    """The stated training set: n scenes of split 0, each labelled by `label_iters` plain FISTA
    iterations from zero, generated and labelled in chunks (snapshots kept on the device, labels
    sparse on the host)."""
    import torch
    ys_all = torch.empty((n, int(mask.sum())), dtype=torch.complex64, device="cuda")
    taus = np.empty(n, dtype=np.float32)
    labels = SparseLabels()
    t0 = time.time()
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        ys, tc = make_split(B, plan, 0, s, e - s, mask)
        ys_all[s:e] = ys
        taus[s:e] = tc
        labels.add_dense_chunk(labels_for(B, plan, ys, tc, label_iters, chunk=chunk))
        print(f"spec data: {e} / {n} scenes labelled ({time.time() - t0:.0f} s, "
              f"{int(np.concatenate(labels.counts).mean())} nonzeros per label)", flush=True)
    labels.finish()
    return ys_all, taus, labels


def train(args):
    import torch
    from . import bccb as B
    from . import scenes as S
    torch.cuda.set_device(0)
    mask = S.learned_fixed_mask()
    plan = B.Plan(mask, 256, 256)
    t0 = time.time()
    if args.spec:
        ys, taus, sparse_labels = spec_data(B, plan, mask, args.train_scenes, args.label_iters)
        labels = None
    else:
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
            sel = np.sort(perm[s:s + args.batch])
            idx = torch.from_numpy(sel).to(ys.device)
            yb = ys.index_select(0, idx).contiguous()
            if labels is None:
                lb = sparse_labels.dense(sel, plan.L, ys.device).reshape(len(sel), plan.L2, plan.L1)
            else:
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
        "labels_stored": "sparse on the host" if args.spec else "dense on the device",
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
    ap.add_argument("--spec", action="store_true",
                    help="the stated training set: 2^20 scenes with 2000-iteration labels, stored sparse "
                         "(sets --train-scenes and --label-iters unless they are given)")
    args = ap.parse_args(argv)
    if args.spec:
        if "--train-scenes" not in (argv or sys.argv):
            args.train_scenes = 1 << 20
        if "--label-iters" not in (argv or sys.argv):
            args.label_iters = 2000
    train(args)


if __name__ == "__main__":
    sys.exit(main())
