"""Train the 3D DeepONet of App. B on non-scattering problems and save the
trained trunk.

Workload (the training configuration): 48^3 grid, homogeneous k ~ U[5, 15],
8-cell sponge, no scatterer, complex Gaussian-random-field sources (length
scale 0.1) scaled to unit RMS.  Labels come from the plain solver (batched
BiCGStab to 1e-8, no network, the standalone Krylov method that also judges
the meta-solver's error); the branch input is the meta-solver's own sampling
of the source (``DON_BRANCH_INPUT``: trilinear onto 16^3, Re then Im, then
k).  Training runs on the library's bf16-MFMA forward/backward kernels with
fp32 master weights and Adam (batch 64, the constant learning rate 1e-4 of
App. B), for whole epochs, until the training loss (mean relative L2 error)
plateaus; the error on a held-out tenth is recorded along the way.

The Krylov meta-solvers use only the trunk: App. C builds the coarse space
from the trunk basis functions evaluated at the grid's nodes.  So the saved
file holds the trunk's layers (fp32, as trained) and the run's record.  Every
numerical step runs in the library; this module only sequences the calls.

    python -m paper_2405_12380_amd.train_deeponet --samples 4096 --max-epochs 3000
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(PKG, "weights", "deeponet_48cube_trunk.npz")
BRANCH_W = [2 * 16 ** 3 + 1, 256, 256, 256, 256, 256]
TRUNK_W = [3, 256, 256, 256, 256, 128]


def log(msg):
    print(f"[train] {msg}", file=sys.stderr, flush=True)


def load_trunk(path: str = DEFAULT_OUT):
    """[(W, b)] float64 layers of a saved trunk, and the run's record."""
    with np.load(path, allow_pickle=False) as z:
        nl = int(z["layers"])
        layers = [(z[f"W{i}"].astype(np.float64), z[f"b{i}"].astype(np.float64)) for i in range(nl)]
        meta = json.loads(str(z["meta"]))
    return layers, meta


def dataset(helm, I, torch, n_samples, n=(48, 48, 48), instance=0, chunk=512, net=None):
    """(ks, F: n_samples x 8193 fp32 branch inputs, Y: n_samples x P complex64
    labels, label-solve record).  Labels by the batched plain BiCGStab to 1e-8,
    ``chunk`` problems per call."""
    P = int(np.prod(n))
    ks, alpha, f = I.config3(n_samples, instance=instance, n=n)
    F = torch.empty((n_samples, BRANCH_W[0]), dtype=torch.float32, device="cuda")
    Y = torch.empty((n_samples, P), dtype=torch.complex64, device="cuda")
    iters, secs, conv = [], 0.0, 0
    for c0 in range(0, n_samples, chunk):
        c1 = min(n_samples, c0 + chunk)
        ops = [helm.Op(n, helm.C128, np.full(P, k * k), alpha, np.zeros(P, np.uint8)) for k in ks[c0:c1]]
        fs = [f[i] for i in range(c0, c1)]
        us = [op.field() for op in ops]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, stats = helm.meta_solve_batch(ops, None, fs, us, kind="bicgstab", tol=1e-8, max_iters=20000)
        torch.cuda.synchronize()
        secs += time.perf_counter() - t0
        iters += [s["iters"] for s in stats]
        conv += sum(s["converged"] for s in stats)
        for j, i in enumerate(range(c0, c1)):
            x = net.branch_input(ops[j], fs[j], k=float(ks[i]))
            F[i] = x.float()
            Y[i] = us[j].to(torch.complex64)
        for op in ops:
            op.close()
        del ops, us, fs
        log(f"labels {c1}/{n_samples}: {secs:.1f} s of solves")
    del f
    rec = {"solves": n_samples, "seconds": round(secs, 2), "iters_min": int(min(iters)), "iters_max": int(max(iters)),
           "converged": int(conv)}
    return ks, F, Y, rec


def train(helm, I, torch, n_samples=4096, max_epochs=3000, patience=100, eval_every=25, seed=0, lr=1e-4,
          batch=64, n=(48, 48, 48), data=None):
    """Train from the seeded Glorot initialisation (App. B: Adam with a
    constant learning rate of 1e-4, until the training loss plateaus);
    returns (net, (branch, trunk) layers, record).  An epoch's training loss
    is the mean of its steps' losses; training stops after ``max_epochs`` or
    once that loss has not improved by 1% for ``patience`` epochs, and the
    final weights are kept.  The validation error (held-out tenth) is recorded
    every ``eval_every`` epochs.  ``data``: a (ks, F, Y, record) tuple from
    ``dataset`` to reuse (labels are solved otherwise)."""
    w = np.random.default_rng([2405, 3, 1 + seed])
    branch = I.glorot_mlp(BRANCH_W, w)
    trunk = I.glorot_mlp(TRUNK_W, w)
    net = helm.DeepONet(helm.C128, branch, trunk, TRUNK_W[-1], head="split_output", branch_grid=(16, 16, 16),
                        k_input=True)
    if data is None:
        log(f"labels: {n_samples} non-scattering {n[0]}^3 solves")
        data = dataset(helm, I, torch, n_samples, n=n, net=net)
        log(f"labels done: {data[3]}")
    ks, F, Y, lrec = data
    n_samples = int(F.shape[0])
    n_val = max(batch, (n_samples // 10) // batch * batch)
    n_train = (n_samples - n_val) // batch * batch
    steps = n_train // batch
    tr = helm.Trainer(net, I.node_points(n), batch=batch, max_steps=max(steps, n_val // batch), lr=lr)
    tr.data(F, Y)
    val_idx = np.arange(n_samples - n_val, n_samples)
    rng = np.random.default_rng([2405, 3, 99, seed])
    hist = [{"epoch": 0, "val": float(tr.eval(val_idx).mean())}]
    log(f"epoch 0: validation {hist[0]['val']:.4f}")
    best_train, best_epoch = np.inf, 0
    t0 = time.perf_counter()
    e = 0
    for e in range(1, max_epochs + 1):
        tl = float(np.mean(tr.steps(rng.permutation(n_train)[:steps * batch])))
        if tl < 0.99 * best_train:
            best_train, best_epoch = tl, e
        stop = e - best_epoch >= patience
        if e % eval_every == 0 or stop or e == max_epochs:
            v = float(tr.eval(val_idx).mean())
            hist.append({"epoch": e, "train": tl, "val": v})
            log(f"epoch {e}: train {tl:.4f} (best {best_train:.4f} at {best_epoch}), validation {v:.4f}, "
                f"{time.perf_counter() - t0:.0f} s")
        if stop:
            break
    train_s = time.perf_counter() - t0
    flat = tr.params()
    bl = tr.unflatten(flat, 0, len(BRANCH_W) - 1)
    tl_layers = tr.unflatten(flat, 1, len(TRUNK_W) - 1)
    tr.export(net)
    tr.close()
    rec = {"samples": n_samples, "train": n_train, "validation": int(n_val), "batch": batch, "lr": lr,
           "epochs_run": e, "plateau_patience": patience, "train_loss_final": hist[-1].get("train"),
           "val_final": hist[-1]["val"], "val_initial": hist[0]["val"], "train_seconds": round(train_s, 1),
           "labels": lrec, "history": hist}
    return net, (bl, tl_layers), rec


def save_trunk(path, trunk_layers, rec):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    arrs = {}
    for i, (W, b) in enumerate(trunk_layers):
        arrs[f"W{i}"] = np.asarray(W, dtype=np.float32)
        arrs[f"b{i}"] = np.asarray(b, dtype=np.float32)
    np.savez_compressed(path, layers=np.int64(len(trunk_layers)), meta=np.array(json.dumps(rec)), **arrs)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--samples", type=int, default=4096)
    ap.add_argument("--max-epochs", type=int, default=3000)
    ap.add_argument("--patience", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_OUT)
    args = ap.parse_args()
    import torch
    from paper_2405_12380_amd import helm, inputs as I
    torch.cuda.set_device(0)
    net, (bl, tl), rec = train(helm, I, torch, args.samples, args.max_epochs, args.patience, seed=args.seed)
    save_trunk(args.out, tl, rec)
    log(f"saved {args.out}: {rec['epochs_run']} epochs, training loss {rec['train_loss_final']:.4f}, "
        f"validation {rec['val_final']:.4f}")
    print(json.dumps({k: v for k, v in rec.items() if k != "history"}))


if __name__ == "__main__":
    main()
