"""Training and use of the warm-start network of the subspace GenEO solver.

Training data come from the method itself: for each training problem the
solver runs the subspace GenEO eigensolver from a random start; its per-dof
features and its converged Ritz vectors (the lowest non-kernel GenEO modes of
every subdomain) are the network's inputs and targets.  Every numerical step
runs in the library's kernels (awg_mlp_* and awg_setup); this module only
moves arrays between them.
"""
from __future__ import annotations

import time

import numpy as np

from . import awg


def collect(workloads, n_targets: int = 4, eig_block: int = 16, eig_tol: float = 1e-10, seed: int = 0,
            log=None) -> list[dict]:
    """Features and target modes of every subdomain of every workload."""
    out = []
    for k, w in enumerate(workloads):
        t0 = time.perf_counter()
        solver = awg.Solver(w.A, w.subs, tau=w.tau, geneo="subspace", eig_block=eig_block, eig_tol=eig_tol,
                            eig_seed=seed + k, coords=w.coords)
        X = solver.export("mlp_features").reshape(-1, awg.MLP_FEATURES)
        Z = solver.export("ritz_vectors")
        sizes = np.array([len(s) for s in w.subs], dtype=np.int64)
        row_ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        tl, off, cols = [], [], []
        o = 0
        for s, n in enumerate(sizes):
            blk = Z[row_ptr[s] * eig_block:(row_ptr[s] + n) * eig_block].reshape(eig_block, n)   # column j = row j
            T = blk[:n_targets]
            nrm = np.linalg.norm(T, axis=1)
            T = T / np.where(nrm > 0, nrm, 1.0)[:, None]
            tl.append(T.astype(np.float32).ravel())                                               # column-major n x m
            off.append(o)
            cols.append(n_targets)
            o += T.size
        out.append(dict(X=X.astype(np.float32), row_ptr=row_ptr, T=np.concatenate(tl), tgt_off=np.array(off, np.int64),
                        tgt_cols=np.array(cols, np.int32), eig_iters=max(solver.stats()["eig_iters"])))
        solver.close()
        if log:
            log(f"collect {k + 1}/{len(workloads)} {w.name} rows={X.shape[0]} {time.perf_counter() - t0:.2f}s")
    return out


def _merge(parts: list[dict]) -> dict:
    X = np.concatenate([p["X"] for p in parts])
    rp, to, tc, T = [0], [], [], []
    roff = toff = 0
    for p in parts:
        rp.extend((p["row_ptr"][1:] + roff).tolist())
        to.extend((p["tgt_off"] + toff).tolist())
        tc.extend(p["tgt_cols"].tolist())
        T.append(p["T"])
        roff += p["X"].shape[0]
        toff += p["T"].size
    return dict(X=X, row_ptr=np.array(rp, np.int64), tgt_off=np.array(to, np.int64), tgt_cols=np.array(tc, np.int32),
                T=np.concatenate(T))


def train(net: "awg.MLP", data: list[dict], steps: int = 400, fields_per_step: int = 4, lr: float = 1e-3,
          ridge: float = 1e-4, seed: int = 0, log=None) -> list[float]:
    """Adam on minibatches of whole training problems; returns the loss per step."""
    import torch
    rng = np.random.default_rng(seed)
    order = []
    hist = []
    dev = torch.device("cuda")
    cache = {}
    for it in range(steps):
        if not order:
            order = list(rng.permutation(len(data)))
        pick = tuple(sorted(order[:fields_per_step]))
        order = order[fields_per_step:]
        if pick not in cache:
            b = _merge([data[i] for i in pick])
            cache = {pick: tuple(torch.as_tensor(b[k], device=dev) for k in ("X", "row_ptr", "tgt_off", "tgt_cols", "T"))}
        X, rp, to, tc, T = cache[pick]
        hist.append(net.loss_grad(X, rp, to, tc, T, ridge))
        net.adam_step(lr=lr)
        if log and (it % 50 == 0 or it == steps - 1):
            log(f"train step {it} loss {hist[-1]:.4f}")
    return hist


def save(net: "awg.MLP", path: str) -> None:
    np.savez(path, dims=np.array(net.dims, np.int64), params=net.get_params())


def load(path: str) -> "awg.MLP":
    with np.load(path, allow_pickle=False) as f:
        dims = [int(v) for v in f["dims"]]
        params = f["params"]
    net = awg.MLP(dims[0], dims[1], len(dims) - 2, dims[-1])
    net.set_params(params)
    return net


# ---------------------------------------------------------------------------
# command line: train a network on seeded synthetic problems, or compare the
# learned and random starts on unseen seeds
#   python -m paper_2106_10913_amd.learned train --family diff3d --m 33 --seeds 1000:1200 --out net.npz
#   python -m paper_2106_10913_amd.learned evaluate --family diff3d --m 65 --seeds 2000:2020 --weights net.npz
# ---------------------------------------------------------------------------
def _workload(family: str, m: int, seed: int):
    import awg_problems as P
    if family == "diff3d":
        nb = max(1, round((m - 1) / 8))
        return P.configs.diff3d_grf(m_cells=m, seed=seed, boxes=(nb, nb, nb))
    if family == "q1_2d":
        return P.q1_2d(m=m, seed=seed)
    raise ValueError(family)


def _seeds(text: str):
    a, b = text.split(":")
    return range(int(a), int(b))


def main(argv=None):
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(prog="python -m paper_2106_10913_amd.learned")
    ap.add_argument("mode", choices=["train", "evaluate"])
    ap.add_argument("--family", default="diff3d", choices=["diff3d", "q1_2d"])
    ap.add_argument("--m", type=int, default=33, help="cells per side")
    ap.add_argument("--seeds", default="1000:1200")
    ap.add_argument("--out", default="net.npz")
    ap.add_argument("--weights", default=None)
    ap.add_argument("--steps", type=int, default=800)
    ap.add_argument("--targets", type=int, default=4)
    ap.add_argument("--channels", type=int, default=8)
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.mode == "train":
        data = []
        for sd in _seeds(args.seeds):
            data.extend(collect([_workload(args.family, args.m, sd)], n_targets=args.targets, seed=sd))
            if len(data) % 20 == 0:
                log(f"collected {len(data)} problems")
        net = awg.MLP(awg.MLP_FEATURES, 256, 3, args.channels, seed=0)
        hist = train(net, data, steps=args.steps, fields_per_step=4, lr=1e-3, log=log)
        save(net, args.out)
        print(json.dumps({"trained_on": f"{args.family} m={args.m} seeds {args.seeds}", "steps": args.steps,
                          "loss_first": hist[0], "loss_last20": float(np.mean(hist[-20:])), "out": args.out}))
        return
    import torch
    net = load(args.weights)
    rows = {"cold": [], "learned": []}
    for sd in _seeds(args.seeds):
        w = _workload(args.family, args.m, sd)
        b = torch.as_tensor(w.b, device="cuda")
        for mode in ("cold", "learned"):
            s = awg.Solver(w.A, w.subs, tau=w.tau, geneo="subspace", coords=w.coords,
                           eig_init=net if mode == "learned" else None)
            st = s.stats()
            _, info = s.pcg(b, tol=w.tol)
            rows[mode].append(dict(it_max=max(st["eig_iters"]), it_mean=float(np.mean(st["eig_iters"])),
                                   fallbacks=st["eig_fallbacks"], geneo_ms=st["ms"]["geneo"],
                                   setup_ms=st["ms"]["total"], n0=st["n0"], pcg_iters=info["iters"],
                                   kappa=info["lmax_est"] / info["lmin_est"]))
            s.close()
        log(f"seed {sd}: it_max cold {rows['cold'][-1]['it_max']} learned {rows['learned'][-1]['it_max']}")
    out = {mode: {k: float(np.mean([r[k] for r in rs])) for k in rs[0]} for mode, rs in rows.items()}
    out["same_n0"] = all(a["n0"] == b["n0"] for a, b in zip(rows["cold"], rows["learned"]))
    out["problems"] = f"{args.family} m={args.m} seeds {args.seeds}"
    print(json.dumps(out))


if __name__ == "__main__":
    main()
