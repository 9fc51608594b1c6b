"""Benchmark: AWG-PCG time to a 1e-8 relative residual (setup + solve) on one
MI355X, FP32 local operators + learned GenEO start against plain FP64.

Default workload (the largest single-GPU configuration, the one the learned
start is built for): 3D Q1 FEM diffusion on 65^3 cells of [0,1]^3, Dirichlet
all round (n = 64^3 = 262,144, nnz = 6,859,000), log10 k = 1.5 x a Gaussian
random field with correlation length U(4,16) cells (seed 2000, a seed the
network never saw), b = ones, 512 boxes of 8^3 nodes with overlap 1, GenEO
threshold tau = 0.1, PCG tolerance 1e-8 on ||r||/||b||.  Synthetic input
shaped like the paper's experiments (no dataset).

One step = awg_setup (every set-up phase on the GPU) + awg_pcg from x0 = 0,
with A, b and the subdomain lists already resident in HBM.  Two forms run
K steps each:
  plain  FP64 everywhere, dense GenEO eigensolver;
  fast   FP32 local operators (eigen-setup, coarse spaces, PCG and W
         recurrences in FP64), subspace GenEO eigensolver warm-started by
         the network, graph-captured PCG iteration.
Both must reach a true residual ||b - A x|| / ||b|| <= 1e-8 in every timed
step (accuracy_ok).  value = the fast form's ms per step; the plain form's
time and the speed-up are reported beside it.  The JSON line also carries
the dominant kernel of the fast form against its roofline and the FP64 CPU
oracle timed on a bounded, phase-by-phase sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
FP16_PEAK_TFLOPS = 2500.0     # dense FP16 matrix cores (no sparsity)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--local-prec", default="f64", choices=["f64", "f32"])
    ap.add_argument("--geneo", default="dense", choices=["dense", "subspace"],
                    help="GenEO eigensolver of the timed FP64 form")
    ap.add_argument("--coarse2", default="ad", choices=["ad", "inex", "hyb"],
                    help="second-coarse-space preconditioner H3 (both forms); ad is the default line")
    ap.add_argument("--h2", default="nn_hyb", choices=["nn_hyb", "asp_hyb", "asp_ad", "as_hyb"],
                    help="two-level preconditioner for A_+ (both forms); nn_hyb is the default line")
    ap.add_argument("--w-h2", default="asp_ad", choices=["asp_ad", "asp_hyb", "nn_hyb"],
                    help="preconditioner of the W solves (with h2 = nn_hyb); nn_hyb is H2 itself")
    ap.add_argument("--w-rtol", type=float, default=1e-10,
                    help="relative residual of the PCG solves for W (the paper's choice is 1e-10)")
    ap.add_argument("--fast-local", default="f32", choices=["f32", "f16x3"],
                    help="local-operator arithmetic of the fast form (f16x3: split-FP16 matrix-core "
                         "local products in the W solves)")
    ap.add_argument("--no-split16", action="store_true",
                    help="skip the extra split-FP16 form reported beside the FP32 fast form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fast-form", action="store_true")
    ap.add_argument("--workload", default="diff3d_64", choices=sorted(WORKLOADS),
                    help="diff3d_64 (the largest single-GPU configuration) is the headline workload")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (HBM counter calibration)")
    return ap.parse_args()


def cpu_baseline(w, workload: str, k_sub: int = 8, b_cols: int = 64):
    """FP64 oracle timed on a bounded, phase-by-phase sample of the workload.

    The oracle's full run on the large workloads takes from many minutes to
    hours, so every phase is timed on a part of the workload and scaled by
    its work ratio to the whole:
      maps     pair counts M_mu and B on k_sub of the N subdomains, x N/k_sub;
      split    eigendecomposition of B^s on k_sub subdomains, x N/k_sub;
      geneo    M_B^s and the generalized eigensolve on the same, x N/k_sub;
      coarse0  E0 = R0 A_+ R0^T for the sampled subdomains' coarse columns,
               x n0/columns, plus the deleting Cholesky of an n0 x n0 Gram
               matrix (n0 estimated as N/k_sub x the sampled columns);
      W        the oracle's route for this size: a sparse LU of A (in full)
               and 2 n_- column solves (sampled on b_cols), or, above
               W_DIRECT_MAX_N, PCG with H2 on every column: it_W x n_-/b_cols x
               (one H2 application to b_cols columns, local parts sampled);
      pcg      iters x (one application of H and one product with A to a
               vector, local parts sampled).
    it_W and iters come from the oracle-only golden file of the workload when
    it holds them (else 40 each), and so do n0 and n_- (else estimated from
    the sample).  Threads: the host cores visible to the
    process (the BLAS uses them all).  Beside the extrapolation, the smallest
    configuration is run by the oracle in full and timed (full_runs).
    """
    import numpy as np
    import scipy.linalg as sla
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    import awg_problems as P
    from oracle import awg_oracle as O
    threads = len(os.sched_getaffinity(0))
    A = w.A.tocsr()
    subs = [np.asarray(t, dtype=np.int64) for t in w.subs]
    n, N = A.shape[0], len(subs)
    k = min(k_sub, N)
    rng = np.random.default_rng(0)
    samp = np.sort(rng.choice(N, k, replace=False))
    scale = N / k
    gold = os.path.join(ROOT, "tests", "golden", f"{workload}.json")
    g = {}
    if os.path.exists(gold):
        with open(gold) as f:
            g = json.load(f)
    iters, it_w, src = 40, 40, "assumed 40"
    if "iters" in g:
        iters, src = int(g["iters"]), "oracle golden file"
        it_w = int(g.get("w_iters_max") or it_w)
    ts = {}
    clock = time.perf_counter
    t0 = clock()
    Ds = O.partition_of_unity(n, subs)
    cnt = O.pair_multiplicity(A, [subs[s] for s in samp])
    ts["maps"] = (clock() - t0) * scale
    # exact M_mu on the rows of the sampled subdomains (untimed input of the
    # sampled phases): counts of subdomains holding both ends of each nonzero,
    # from the subdomain incidence matrix S (N x n) as (S^T S)_ij on A's pattern
    S = sp.csr_matrix((np.ones(sum(t.size for t in subs)),
                       (np.concatenate([np.full(t.size, q) for q, t in enumerate(subs)]), np.concatenate(subs))),
                      shape=(N, n))
    rows = np.unique(np.concatenate([subs[s] for s in samp]))
    C = (S[:, rows].T @ S).tocsr()
    Ar = A[rows]
    cnt = np.maximum(np.asarray(C[np.repeat(np.arange(rows.size), np.diff(Ar.indptr)), Ar.indices]).ravel(), 1)
    Bd = A.tolil()
    Bd[rows] = sp.csr_matrix((Ar.data / cnt, Ar.indices, Ar.indptr), shape=Ar.shape)
    B = Bd.tocsr()
    empty = O.LocalSplit(np.zeros(0), np.zeros((0, 0)), 0, 0, 0.0)
    split = [empty] * N
    t0 = clock()
    for s in samp:
        split[s] = O.split_local(O.local_block(B, subs[s]))
    ts["split"] = (clock() - t0) * scale
    Ys = {}
    t0 = clock()
    for s in samp:
        Ys[s], _ = O.geneo_local(split[s], Ds[s], O.local_MB(A, subs, split, s), w.tau)
    ts["geneo"] = (clock() - t0) * scale
    # coarse0: the sampled columns of R0^T through A_+ and R0
    rows_, cols_, vals_ = [], [], []
    off = 0
    for s in samp:
        m = Ys[s].shape[1]
        rows_.append(np.repeat(subs[s], m))
        cols_.append(np.tile(np.arange(off, off + m), subs[s].size))
        vals_.append(Ys[s].ravel())
        off += m
    R0T = sp.csr_matrix((np.concatenate(vals_), (np.concatenate(rows_), np.concatenate(cols_))), shape=(n, off))
    n0 = int(g["n0"]) if "n0" in g else max(1, int(round(off * scale)))
    st = O.AWGSetup(A=A, subs=subs, tau=w.tau, Ds=Ds, cnt=cnt, B=B, split=split, Y=None, geneo_lam=None,
                    R0T=R0T, E0=None, E0_cho=None, W=np.zeros((n, 0)), EW=None, EW_cho=None, Vg=None, w_info={})
    t0 = clock()
    _ = R0T.T.tocsr() @ st.A_plus_mv(R0T.toarray())
    t_cols = clock() - t0
    Gm = rng.standard_normal((n0, n0 + 8))
    G = Gm @ Gm.T
    t0 = clock()
    O.gram_keep(G)
    Gc = sla.cho_factor(G, lower=True)
    ts["coarse0"] = t_cols * n0 / max(1, off) + (clock() - t0)
    nm = int(g["n_minus"]) if "n_minus" in g else max(1, int(round(sum(split[s].nstrict for s in samp) * scale)))

    def apply_local(X):
        """local parts of one application (A_- and H^NN) on the sampled subdomains"""
        for s in samp:
            sp_ = split[s]
            Xs = Ds[s][:, None] * X[subs[s]]
            sp_.V_minus @ (sp_.V_minus.T @ Xs)
            sp_.V_plus @ ((sp_.V_plus.T @ Xs) / sp_.L_plus[:, None])

    def h2_cost(b):
        """seconds of one oracle H2 application to b columns (+ one A_+ product)"""
        X = rng.standard_normal((n, b))
        t0 = clock()
        apply_local(X)
        t_loc = (clock() - t0) * scale * 2              # H^NN and the two A_- terms of H2 and A_+
        t0 = clock()
        for _ in range(3):
            A @ X                                        # two A_+ products in H2, one in PCG
        u = sla.cho_solve(Gc, rng.standard_normal((n0, b)))
        sla.cho_solve(Gc, u)                             # two E0 solves
        t_glob = clock() - t0
        t0 = clock()
        for _ in range(2):                               # two R0 and two R0^T products (sampled columns)
            R0T @ u[:off]
            R0T.T @ X
        return t_loc + t_glob + (clock() - t0) * n0 / max(1, off)

    if n <= O.W_DIRECT_MAX_N:
        t0 = clock()
        lu = spla.splu(A.tocsc())
        t_lu = clock() - t0
        V = np.zeros((n, b_cols))
        V[rng.integers(0, n, b_cols), np.arange(b_cols)] = 1.0
        t0 = clock()
        lu.solve(V)
        ts["W"] = t_lu + (clock() - t0) * 2 * nm / b_cols
        w_how = f"sparse LU of A in full ({t_lu:.1f} s) + {b_cols} of 2 n_- column solves"
    else:
        ts["W"] = it_w * (nm / b_cols) * h2_cost(b_cols)
        w_how = f"PCG with H2: {it_w} iterations x n_-/{b_cols} x one H2 application to {b_cols} columns"
    Wr = rng.standard_normal((n, min(nm, 512)))
    t0 = clock()
    Wr.T @ (A @ Wr)
    ts["W"] += (clock() - t0) * (nm / Wr.shape[1]) ** 2       # E_W = W^T A W
    r = rng.standard_normal(n)
    t0 = clock()
    Wr @ (Wr.T @ r)
    t_w = (clock() - t0) * nm / Wr.shape[1]
    ts["pcg"] = iters * (h2_cost(1) + t_w)
    total = sum(ts.values())
    # the smallest configuration (32x32 five-point diffusion, 16 subdomains)
    # run by the oracle in full (set-up and PCG), timed in the same run
    full = []
    for label, make in (("fd5_32 (n = 1024, 16 subdomains)", P.fd5_32),):
        ws = make()
        t0 = clock()
        sts = O.setup(ws.A, ws.subs, ws.tau)
        t_set = clock() - t0
        t0 = clock()
        res = O.pcg(ws.A, ws.b, sts.apply, tol=ws.tol, maxit=1000)
        full.append({"workload": label, "setup_s": round(t_set, 3), "pcg_s": round(clock() - t0, 3),
                     "iters": res.iters, "n": int(ws.A.shape[0])})
    return {
        "value": round(total * 1e3, 1), "unit": "ms", "cores": threads, "kind": "oracle",
        "full_runs": full,
        "sample": (f"extrapolated from a bounded sample, not a full run: maps, B^s splitting and GenEO on "
                   f"{k} of {N} subdomains (x{N}/{k}); E0 columns of those subdomains (x n0/{off}, n0 = {n0}) "
                   f"+ the deleting Cholesky of an {n0}^2 Gram matrix; W ({nm} columns est.): {w_how}; "
                   f"E_W by its GEMMs on 512 columns; PCG: {iters} iterations ({src}) x one application "
                   f"with the local parts sampled"),
        "phases_s": {k_: round(v, 2) for k_, v in ts.items()},
    }


# kernels whose roofline is the matrix cores (FP64 MFMA); every other
# instrumented kernel is HBM bound
MFMA_KERNELS = ("k_gemm",)

# HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE
# (two runs), each scaled by what the counter reads for a plain 1 GiB copy
# (factors 2.0 and 1.0).  Valid only for the kernel source and workload they
# were taken on; otherwise the bench reports traffic = null.
TRAFFIC = {
    "k_gemm128_f32_w8:P": {
        # FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (copy calibration) summed over
        # the launches of one timed step (widths b = 1652 x 32, 944, 418,
        # 166 x 2, 16 x 2); per launch = this / the step's launch count (the
        # tuner may run the two b = 16 launches, 0.25 % of the bytes, in the
        # persistent variant instead)
        "bytes_per_step": 1.7438e12,
        "source": "paper_2106_10913_amd/csrc/k_dense.hip",
        "sha256": "5c0d19796b853ef1bb1de4d0fb4c14e5f643733b8a350e70b968f4a873fd59e5",
        "workload": "q1_diffusion_64^3_grf_box8^3_overlap1_tau0.1",
    },
}


def measured_traffic(name: str, workload: str, calls_per_step: float):
    import hashlib
    rec = TRAFFIC.get(name)
    if rec is None or rec["workload"] != workload or calls_per_step <= 0:
        return None
    with open(os.path.join(ROOT, rec["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["sha256"]:
            return None
    return rec["bytes_per_step"] / calls_per_step


def kernel_rates(kt: dict, top: int = 20) -> dict:
    """Achieved rate of each instrumented kernel over the warm-up step: HBM
    kernels as algorithmic GB/s and fraction of the HBM peak, MFMA kernels as
    TFLOP/s and fraction of the FP64 peak (FP32 for the FP32 local product,
    FP16 for the split-FP16 one).
    """
    out = {}
    for name, rec in sorted(kt.items(), key=lambda kv: -kv[1]["ms"])[:top]:
        if name.startswith("graph:") or rec["ms"] <= 0:
            continue
        if name.startswith(MFMA_KERNELS) and rec["flops"] > 0:
            peak = (FP16_PEAK_TFLOPS if "_h3" in name else
                    FP32_PEAK_TFLOPS if ("_mix" in name or "_f32" in name) else FP64_PEAK_TFLOPS)
            tf = rec["flops"] / (rec["ms"] * 1e-3) / 1e12
            out[name] = {"TFLOP/s": round(tf, 2), "frac": round(tf / peak, 3), "calls": rec["calls"]}
        elif rec["bytes"] > 0:
            gbs = rec["bytes"] / (rec["ms"] * 1e-3) / 1e9
            out[name] = {"GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 3), "calls": rec["calls"]}
    return out


def roofline(kt: dict, steps: int, workload: str) -> dict:
    """Roofline of the dominant kernel (largest total time in the warm-up step),
    timed live in the timed steps: achieved = its algorithmic bytes (or flops)
    summed over its launches / their summed duration (HIP events recorded by
    the library on its own stream around each launch).
    """
    kernels = {k: v for k, v in kt.items() if not k.startswith("graph:")}
    name, rec = max(kernels.items(), key=lambda kv: kv[1]["ms"])
    avg_us = rec["ms"] * 1e3 / rec["calls"]
    if name.startswith(MFMA_KERNELS):
        achieved = rec["flops"] / (rec["ms"] * 1e-3) / 1e12
        f32 = "_mix" in name or "_f32" in name
        f16 = "_h3" in name
        # the split-FP16 product counts its algorithmic flops once (three
        # FP16 MFMA products are issued per product term) against the FP16 peak
        peak = FP16_PEAK_TFLOPS if f16 else (FP32_PEAK_TFLOPS if f32 else FP64_PEAK_TFLOPS)
        dtype = "f16x3" if f16 else ("f32" if f32 else "f64")
        out = {"kernel": name, "bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
               "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "dtype": dtype,
               "traffic": measured_traffic(name, workload, rec["calls"] / steps),
               "calls_per_step": rec["calls"] / steps, "avg_launch_us": round(avg_us, 2),
               "flops_per_launch": rec["flops"] / rec["calls"]}
        if dtype == "f64":
            # the device's sustained FP64 matrix-core rate (register-only MFMA
            # chains, no memory traffic), measured in this run beside the
            # published peak
            from paper_2106_10913_amd import awg
            sustained = awg.probe_mfma_f64()
            out["sustained_mfma_peak"] = round(sustained, 2)
            out["frac_of_sustained"] = round(achieved / sustained, 4)
        return out
    achieved = rec["bytes"] / (rec["ms"] * 1e-3) / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(name, workload, rec["calls"] / steps),
            "calls_per_step": rec["calls"] / steps,
            "avg_launch_us": round(avg_us, 2), "bytes_per_launch": rec["bytes"] / rec["calls"]}


# workload name -> (generator, config string, network file of its family or None)
def _q1_2d_256(P):
    return P.q1_2d(m=256)


def _q1_2d_512_rcb(P):
    return P.q1_2d(m=512, seed=2, partition="rcb", nparts=256, delta=2)


def _elast3d_40(P):
    return P.configs.elast3d(40)


def _diff3d_64(P):
    return P.configs.diff3d_grf(65, seed=2000)


WORKLOADS = {
    "q1_2d_256": (_q1_2d_256, "q1_2d_diffusion_256x256_box8x8_overlap2_tau0.1", "geneo_q1_2d.npz"),
    "q1_2d_512_rcb": (_q1_2d_512_rcb, "q1_2d_diffusion_512x512_rcb256_overlap2_tau0.1", "geneo_q1_2d.npz"),
    "elast3d_40": (_elast3d_40, "q1_elasticity_40^3_spheres10pct_box8^3_overlap1_tau0.05", None),
    "diff3d_64": (_diff3d_64, "q1_diffusion_64^3_grf_box8^3_overlap1_tau0.1", "geneo_diff3d.npz"),
}


def make_workload(name: str):
    import awg_problems as P
    return WORKLOADS[name][0](P)


def copy_probe(torch, mib: int) -> None:
    """Plain copy kernel of known size: reads and writes mib MiB per launch."""
    n = mib * (1 << 20) // 8
    src = torch.rand(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.add(src, 0.0, out=dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": 3}))


def setup_work(w, st) -> dict:
    """Algorithmic set-up flops of one step: per subdomain n_s^3/3 (Cholesky of
    K^s) + n_s^3/3 (Cholesky of M_B^s) + n_s^3 (the dense transforms) +
    it_eig 2 n_s^2 b (subspace GenEO iterations, b columns), then
    it_W n_- [2 sum n_s^2 + 3 . 2 nnz + 8 sum n_s k_s + 8 sum n_s m_s] for the
    W solves, 2 n n_-^2 for E_W and (n0^3 + n_-^3)/3 for the coarse
    factorisations.  Of these, the W local products 2 sum n_s^2 n_- it_W run
    on FP32 matrix cores in the fast form."""
    import numpy as np
    ns = np.array([len(t) for t in w.subs], dtype=np.float64)
    ks = np.array(st["k_s"], dtype=np.float64)
    ms = np.array(st["m_s"], dtype=np.float64)
    nnz, n = float(w.A.nnz), float(w.A.shape[0])
    nm, n0, itw = float(st["n_minus"]), float(st["n0"]), float(st["w_iters"])
    it_eig = float(max(st["eig_iters"], default=0))
    local = float(np.sum(ns ** 3 / 3 * 2 + ns ** 3 + it_eig * 2 * ns ** 2 * st.get("eig_block", 16)))
    w_local = itw * nm * 2 * float(np.sum(ns ** 2))
    w_rest = itw * nm * (6 * nnz + 8 * float(np.sum(ns * ks)) + 8 * float(np.sum(ns * ms)))
    coarse = 2 * n * nm ** 2 + (n0 ** 3 + nm ** 3) / 3
    return {"local": local, "w_local_product": w_local, "w_rest": w_rest, "coarse": coarse,
            "total": local + w_local + w_rest + coarse}


def form_result(infos, tol):
    """Accuracy of the timed steps of one form: every step must have converged
    with a true residual <= tol."""
    ok = all(i["converged"] == 1 and i["rel_res_true"] <= tol for i in infos)
    return ok, max(i["rel_res_true"] for i in infos)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    if args.copy_probe:
        copy_probe(torch, args.copy_probe)
        return
    from paper_2106_10913_amd import awg
    from paper_2106_10913_amd import learned

    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    w = make_workload(args.workload)
    print(f"# workload {args.workload}: n={w.A.shape[0]} nnz={w.A.nnz} N={len(w.subs)} "
          f"(generated in {time.perf_counter() - t_gen:.1f} s)", file=sys.stderr, flush=True)
    A = w.A
    sizes = np.array([len(s) for s in w.subs], dtype=np.int64)
    ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    idx = np.concatenate(w.subs).astype(np.int32)
    Ad = (torch.as_tensor(A.indptr.astype(np.int64), device=dev),
          torch.as_tensor(A.indices.astype(np.int32), device=dev),
          torch.as_tensor(A.data.astype(np.float64), device=dev))
    Sd = (torch.as_tensor(ptr, device=dev), torch.as_tensor(idx, device=dev))
    bd = torch.as_tensor(w.b, device=dev)
    x = torch.empty_like(bd)
    coords = torch.as_tensor(w.coords, device=dev)
    wfile = WORKLOADS[args.workload][2]
    net = learned.load(os.path.join(ROOT, "paper_2106_10913_amd", "weights", wfile)) if wfile else None

    def step(local_prec, geneo, init):
        t0 = time.perf_counter()
        solver = awg.Solver(Ad, Sd, tau=w.tau, local_prec=local_prec, geneo=geneo, eig_init=init,
                            coords=coords if init is not None else None, coarse2=args.coarse2,
                            w_rtol=args.w_rtol, h2=args.h2, w_h2=args.w_h2)
        t1 = time.perf_counter()
        _, info = solver.pcg(bd, tol=w.tol, maxit=1000, x=x)
        st = solver.stats()
        t2 = time.perf_counter()
        solver.close()
        torch.cuda.synchronize()
        st["wall_ms"] = {"setup": (t1 - t0) * 1e3, "pcg": (t2 - t1) * 1e3, "close": (time.perf_counter() - t2) * 1e3}
        return info, st

    def run_form(label, local_prec, geneo, init, time_dominant):
        """Warm-up steps (the autotuner measures its variants there), one
        untimed step with every kernel instrumented (per-kernel breakdown of
        a step, dominant kernel), then the timed steps; with time_dominant
        the HIP events stay on around the dominant kernel only (per-launch
        events cost microseconds of host time each)."""
        awg.kernel_timing_filter("")
        awg.kernel_timing(False)
        for i in range(max(1, args.warmup)):
            info, st = step(local_prec, geneo, init)
            print(f"# {label} warmup {i}: iters={info['iters']} true_res={info['rel_res_true']:.2e} "
                  f"setup_ms={st['ms']['total']:.1f}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        awg.kernel_times(reset=True)
        awg.kernel_timing(True)
        step(local_prec, geneo, init)
        torch.cuda.synchronize()
        awg.kernel_timing(False)
        kt_warm = awg.kernel_times(reset=True)
        dominant = max((k for k in kt_warm if not k.startswith("graph:")), key=lambda k: kt_warm[k]["ms"])
        if time_dominant:
            awg.kernel_timing_filter(dominant)
            awg.kernel_timing(True)
        infos, stats = [], []
        t0 = time.perf_counter()
        step_ms = []
        for i in range(args.steps):
            ts = time.perf_counter()
            info, st = step(local_prec, geneo, init)
            step_ms.append((time.perf_counter() - ts) * 1e3)
            infos.append(info)
            stats.append(st)
            wm = st["wall_ms"]
            print(f"# {label} step {i}: {step_ms[-1]:.1f} ms (set-up {wm['setup']:.1f}, phases "
                  f"{st['ms']['total']:.1f}, W {st['ms'].get('second_coarse_W', 0.0):.1f} (alloc "
                  f"{st['ms'].get('alloc:second_coarse_W', 0.0):.1f}), coarse0 {st['ms'].get('coarse0', 0.0):.1f} "
                  f"(alloc {st['ms'].get('alloc:coarse0', 0.0):.1f}), pcg {wm['pcg']:.1f}, "
                  f"close {wm['close']:.1f}) iters={info['iters']} converged={info['converged']} "
                  f"true_res={info['rel_res_true']:.2e}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        awg.kernel_timing(False)
        awg.kernel_timing_filter("")
        kt = {k: v for k, v in awg.kernel_times(reset=True).items() if k == dominant}
        ok, worst = form_result(infos, w.tol)
        st, info = stats[-1], infos[-1]
        wk = setup_work(w, st)
        # time the set-up would take with every flop at its matrix-core peak
        # (the W local products at the FP32 peak in the FP32 form, at a third
        # of the FP16 peak in the split-FP16 form: three products per term)
        lp_peak = {"f32": FP32_PEAK_TFLOPS, "f16x3": FP16_PEAK_TFLOPS / 3.0}.get(local_prec)
        t_peak = ((wk["total"] - (wk["w_local_product"] if lp_peak else 0.0)) / (FP64_PEAK_TFLOPS * 1e12)
                  + (wk["w_local_product"] / (lp_peak * 1e12) if lp_peak else 0.0))
        rec = {"ms_per_step": round(ms, 3), "step_ms": [round(v, 1) for v in step_ms],
               "step_phases_ms": [{k: round(v, 1) for k, v in s_["ms"].items()} for s_ in stats],
               "step_eig_fallbacks": [s_["eig_fallbacks"] for s_ in stats],
               "accuracy_ok": ok, "worst_true_res": worst,
               "setup_roofline": {"flops": wk, "setup_ms": round(st["ms"]["total"], 3),
                                  "ms_at_peak": round(t_peak * 1e3, 3),
                                  "frac": round(t_peak * 1e3 / st["ms"]["total"], 4)},
               "local_prec": local_prec, "geneo": geneo, "iters": info["iters"],
               "restarts": info.get("restarts", 0),
               "kappa_est": info["lmax_est"] / info["lmin_est"], "n_minus": st["n_minus"], "n0": st["n0"],
               "w_iters": st["w_iters"], "w_iters_mean": st.get("w_iters_mean"),
               "w_compactions": st.get("w_compactions"),
               "w_factor_fp64_fallbacks": st.get("w_factor_fallbacks"),
               "eig_fallbacks": st["eig_fallbacks"], "eig_learned": st["eig_learned"],
               "eig_iters_max": max(st["eig_iters"], default=0),
               "phases_ms": {k: round(v, 3) for k, v in st["ms"].items()},
               "kernels_ms_per_step": {k: round(v["ms"], 3) for k, v in
                                       sorted(kt_warm.items(), key=lambda kv: -kv[1]["ms"])[:16]},
               "kernel_rates": kernel_rates(kt_warm, top=16)}
        return rec, kt, dominant

    fast_only = args.local_prec == "f32"
    plain = None
    if not fast_only:
        plain, _, _ = run_form("plain", "f64", args.geneo, None, time_dominant=False)
    fast = split16 = None
    if not args.no_fast_form:
        # FP32 local operators, the subspace GenEO solver and the learned start
        # (the two-pencil coarse space of as_hyb has the dense GenEO solver only)
        fgeneo, fnet = ("dense", None) if args.h2 == "as_hyb" else ("subspace", net)
        fast, kt, dominant = run_form("fast", args.fast_local, fgeneo, fnet, time_dominant=True)
        fast["network"] = wfile if fnet is not None else None
        head, head_label = fast, "fast"
        if args.fast_local == "f32" and not args.no_split16:
            # the same form with the W solves' local products on split-FP16
            # matrix cores, reported beside the headline (not the headline:
            # the metric names FP32 local operators)
            split16, _, _ = run_form("split16", "f16x3", fgeneo, fnet, time_dominant=False)
    else:
        plain, kt, dominant = run_form("plain", "f64", args.geneo, None, time_dominant=True)
        head, head_label = plain, "plain"
    out = {
        "metric": "AWG-PCG time to 1e-8 rel. residual (setup+solve), FP32/learned vs plain FP64",
        "value": head["ms_per_step"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f64+" + args.fast_local + "local") if head_label == "fast" else "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload][1], "form": head_label,
                   "n": int(A.shape[0]), "nnz": int(A.nnz), "N": len(w.subs), "tol": w.tol,
                   "coarse2": args.coarse2, "h2": args.h2, "w_h2": args.w_h2 if args.h2 == "nn_hyb" else args.h2,
                   "w_rtol": args.w_rtol},
        "accuracy_ok": head["accuracy_ok"] and (plain is None or plain["accuracy_ok"]),
    }
    if plain is not None and head is not plain:
        out["plain_f64"] = plain
        out["speedup_vs_f64"] = (round(plain["ms_per_step"] / head["ms_per_step"], 3)
                                 if out["accuracy_ok"] else None)
    out[head_label + "_form"] = head
    if split16 is not None:
        out["f16x3_form"] = split16
        out["f16x3_speedup_vs_f64"] = (round(plain["ms_per_step"] / split16["ms_per_step"], 3)
                                       if plain is not None and split16["accuracy_ok"] else None)
    out["roofline"] = roofline(kt, args.steps, out["config"]["workload"])
    out["autotune"] = {k: v["variant"] for k, v in awg.tune_report().items()}
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(w, args.workload)
        print(f"# cpu baseline sample took {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
