"""Training and use of the learned per-aggregate weights.

Targets come from convergence factors the method measures itself: for each
sampled coefficient field (the 2D lognormal, gamma = 5 family at 64^2 nodes),
every pair (omega_P, omega_S) of a small grid builds a hierarchy with those
uniform weights and the library's probe estimates its asymptotic convergence
factor; the pair with the smallest factor is the field's target and every
aggregate of that field's hierarchy contributes one feature row with that
target.  The network is trained on the GPU by the library's own forward,
gradient and Adam kernels (bfloat16 matrix cores, FP32 master weights).

Weights file: JSON with the 5122 parameters, the feature normalisation, the
training seeds and the loss history.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

from . import mbamg
from .inputs import WORKLOADS, make_system

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "mlp_2d64_lognormal.json")
# trained on 2000 fields of varying contrast and coupling (2d-64-mixed); adapts
# per field on 2D systems but does not carry over to 3D coarse levels
MIXED_WEIGHTS = os.path.join(HERE, "weights", "mlp_2d64_mixed.json")
OMEGA_P_GRID = (0.0, 1.0 / 3.0, 0.5, 2.0 / 3.0, 5.0 / 6.0)
OMEGA_S_GRID = (0.5, 0.6, 0.7, 0.8, 0.9, 1.0, 1.1)
TRAIN_FAMILY = "2d-64-lognormal"


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def family_kwargs(family: str, seed: int) -> dict:
    """Generator arguments of one sampled field.  "2d-64-mixed" (64^2 nodes)
    draws the lognormal contrast sigma in [0.25, 2] and the coupling strength
    gamma log-uniformly in [0.3, 10] per field (from the field's seed); any
    other name is a fixed workload."""
    if family == "2d-64-mixed":
        u = np.random.default_rng([int(seed), 7]).random(2)
        return dict(n=64, dim=2, kappa="lognormal", sigma=float(0.25 + 1.75 * u[0]),
                    gamma=float(np.exp(np.log(0.3) + (np.log(10.0) - np.log(0.3)) * u[1])))
    return dict(WORKLOADS[family])


def label_field(seed: int, family: str = TRAIN_FAMILY, probe_iters: int = 10):
    """Best uniform (omega_P, omega_S) of one field by probe, and the feature
    rows of the hierarchy built with it."""
    kw = family_kwargs(family, seed)
    s = make_system(seed=seed, **kw)
    blocks = mbamg.to_device(s)
    best = (np.inf, 0.0, 0.8)
    table = np.zeros((len(OMEGA_P_GRID), len(OMEGA_S_GRID)))
    for a, wp in enumerate(OMEGA_P_GRID):
        h = mbamg.Hierarchy(blocks, s.dofs, s.n_vec, omega_p=wp)
        for b, ws in enumerate(OMEGA_S_GRID):
            h.set_omega(ws)
            rho = h.probe(probe_iters, seed)
            rho = rho if np.isfinite(rho) else 10.0
            table[a, b] = rho
            if rho < best[0]:
                best = (rho, wp, ws)
        h.close()
    _, wp, ws = best
    h = mbamg.Hierarchy(blocks, s.dofs, s.n_vec, judge=0,
                        weights=lambda l, n, F: (np.full(n, wp), np.full(n, ws)))
    rows = [h.features(l) for l in range(h.num_levels() - 1)]
    h.close()
    X = np.concatenate(rows, axis=0)
    T = np.tile(np.array([wp, ws], dtype=np.float32), (X.shape[0], 1))
    return X, T, table


def _save_data(path, Xs, Ts, tables, seeds):
    # compact: features in float16, one target per field
    counts = np.array([x.shape[0] for x in Xs], dtype=np.int32)
    np.savez_compressed(path, X=np.concatenate(Xs).astype(np.float16), counts=counts,
                        targets=np.stack([t[0] for t in Ts]), tables=np.stack(tables), seeds=np.asarray(seeds))


def load_data(path):
    d = np.load(path)
    X = d["X"].astype(np.float32)
    T = np.repeat(d["targets"], d["counts"], axis=0).astype(np.float32)
    return X, T, d["tables"], d["seeds"]


def collect(seeds, out_path=None, progress_every=50, family=TRAIN_FAMILY):
    Xs, Ts, tables = [], [], []
    t0 = time.time()
    for k, seed in enumerate(seeds):
        X, T, table = label_field(int(seed), family)
        Xs.append(X)
        Ts.append(T)
        tables.append(table)
        if (k + 1) % progress_every == 0 or k + 1 == len(seeds):
            _log(f"[learned] labelled {k + 1}/{len(seeds)} fields in {time.time() - t0:.1f} s")
            if out_path and ((k + 1) % (progress_every * 10) == 0 or k + 1 == len(seeds)):
                _save_data(out_path, Xs, Ts, tables, seeds[:k + 1])
    return np.concatenate(Xs), np.concatenate(Ts), np.stack(tables)


def train(X, T, epochs=40, batch=8192, lr=1e-3, seed=0, init=None):
    """Adam on the GPU with the library's kernels; returns (params, mean, std, history)."""
    import torch
    mean = X.mean(axis=0).astype(np.float32)
    std = X.std(axis=0).astype(np.float32)
    std[std < 1e-6] = 1.0
    Xn = ((X - mean) / std).astype(np.float32)
    dev = torch.device("cuda")
    Xd = torch.from_numpy(Xn).to(dev)
    Td = torch.from_numpy(np.ascontiguousarray(T, dtype=np.float32)).to(dev)
    if init is None:
        rng = np.random.default_rng(seed)
        th = np.concatenate([rng.standard_normal(768) * np.sqrt(2.0 / 12), np.zeros(64),
                             rng.standard_normal(4096) * np.sqrt(2.0 / 64), np.zeros(64),
                             rng.standard_normal(128) * 0.01, np.zeros(2)]).astype(np.float32)
    else:
        th = np.asarray(init, dtype=np.float32)
    P = torch.from_numpy(th).to(dev)
    G = torch.zeros_like(P)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    L = torch.zeros(1, dtype=torch.float32, device=dev)
    n = Xd.shape[0]
    rng = np.random.default_rng(seed + 1)
    hist = []
    step = 0
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(n)).to(dev)
        tot = 0.0
        for b0 in range(0, n, batch):
            idx = order[b0:b0 + batch]
            xb = Xd.index_select(0, idx).contiguous()
            tb = Td.index_select(0, idx).contiguous()
            mbamg.mlp_loss_grad(P, xb, tb, G, L)
            step += 1
            mbamg.mlp_adam(P, G, M, V, step, lr=lr)
            tot += float(L.item()) * xb.shape[0]
        hist.append(tot / n)
        if ep % 5 == 0 or ep == epochs - 1:
            _log(f"[learned] epoch {ep}: loss {hist[-1]:.5f}")
    return P.cpu().numpy(), mean, std, hist


def save(path, params, mean, std, meta):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    doc = dict(meta)
    doc.update({"format": "mbamg-mlp-1", "n_params": 5122, "params": [float(v) for v in params],
                "feature_mean": [float(v) for v in mean], "feature_std": [float(v) for v in std]})
    with open(path, "w") as f:
        json.dump(doc, f)


def load(path=DEFAULT_WEIGHTS) -> np.ndarray:
    """5146 floats: parameters, feature means, feature stds (the layout the C-ABI takes)."""
    with open(path) as f:
        doc = json.load(f)
    return np.concatenate([np.asarray(doc["params"], dtype=np.float32),
                           np.asarray(doc["feature_mean"], dtype=np.float32),
                           np.asarray(doc["feature_std"], dtype=np.float32)])


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="label fields and train the per-aggregate weight network")
    ap.add_argument("--fields", type=int, default=2000)
    ap.add_argument("--seed0", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--data", default=None, help="npz of labelled rows to write, or comma-separated npz files to reuse")
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--family", default=TRAIN_FAMILY, help="field family: a workload name or 2d-64-mixed")
    a = ap.parse_args(argv)
    import torch
    mbamg.lib()
    torch.cuda.set_device(0)
    seeds = list(range(a.seed0, a.seed0 + a.fields))
    if a.data and all(os.path.exists(d) for d in a.data.split(",")):
        parts = [load_data(d) for d in a.data.split(",")]
        X = np.concatenate([p[0] for p in parts])
        T = np.concatenate([p[1] for p in parts])
        tables = np.concatenate([p[2] for p in parts])
        sets = [{"data": os.path.basename(d), "fields": int(len(p[3])), "seeds": [int(p[3].min()), int(p[3].max())]}
                for d, p in zip(a.data.split(","), parts)]
        _log(f"[learned] reusing {X.shape[0]} rows from {a.data}")
    else:
        X, T, tables = collect(seeds, a.data, family=a.family)
        sets = [{"family": a.family, "fields": len(seeds), "seeds": [seeds[0], seeds[-1]]}]
    params, mean, std, hist = train(X, T, epochs=a.epochs)
    best = [(OMEGA_P_GRID[int(i) // len(OMEGA_S_GRID)], OMEGA_S_GRID[int(i) % len(OMEGA_S_GRID)])
            for i in np.argmin(tables.reshape(tables.shape[0], -1), axis=1)]
    save(a.out, params, mean, std, {
        "train_family": a.family, "train_sets": sets,
        "rows": int(X.shape[0]), "omega_p_grid": list(OMEGA_P_GRID), "omega_s_grid": list(OMEGA_S_GRID),
        "probe_iters": 10, "epochs": a.epochs, "loss_history": hist,
        "target_counts": {f"{wp:.3f},{ws:.2f}": best.count((wp, ws)) for wp, ws in sorted(set(best))}})
    _log(f"[learned] wrote {a.out}")


if __name__ == "__main__":
    main()
