"""Train the warm-start U-Net on solver-generated fields and save its weights.

    python -m paper_2412_00031_amd.train_warmstart --models 100 --src 20 --epochs 12

Fields: converged forward solves (tol 1e-6) on random smooth models of the
101^3 spherical geometry (0-100 km depth, 4 x 4 deg), sampled on every second
node (51^3, padded to 56^3).  Writes paper_2412_00031_amd/weights/unet_sph101.npz
with the parameters and the training record.
"""
import argparse
import json
import sys
import time

import numpy as np
import torch

from . import workloads as W
from .warmstart import WEIGHTS, UNet, build_training_set, train


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--models", type=int, default=100)
    ap.add_argument("--src", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=9001)
    ap.add_argument("--out", default=WEIGHTS)
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("training needs a GPU")
    log = lambda m: print(m, flush=True)
    grid = W.spherical_grid(101, 100.0, 2.0)
    t0 = time.time()
    data = build_training_set(grid, a.models, a.src, a.seed, log=log)
    torch.cuda.synchronize()
    t_data = time.time() - t0
    log(f"training set: {a.models * a.src} fields in {t_data:.1f} s")
    net = UNet("cuda", seed=a.seed)
    t1 = time.time()
    hist = train(net, data, a.epochs, batch=a.batch, lr=a.lr, seed=a.seed, log=log)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    record = dict(models=a.models, src_per_model=a.src, epochs=a.epochs, batch=a.batch, lr=a.lr, seed=a.seed,
                  data_s=round(t_data, 1), train_s=round(t_train, 1),
                  history=[[int(e), float(tl), float(vl)] for e, tl, vl in hist],
                  mean_iters_plain=float(np.mean(np.abs(data["iters"]))))
    net.save(a.out, record=json.dumps(record))
    log(json.dumps(record))


if __name__ == "__main__":
    main()
