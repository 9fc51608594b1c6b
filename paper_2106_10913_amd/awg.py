"""ctypes binding of libawg (include/awg.h).

Argument marshalling only: every step of the set-up, the preconditioner and
PCG runs in the HIP library.  PyTorch provides device memory and the stream.
The binding refuses to run when the library has not been built.
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libawg.so")

AWG_LOCAL_F64 = 0
AWG_LOCAL_F32 = 1
AWG_LOCAL_F16X3 = 2
LOCAL_PREC = {"f64": AWG_LOCAL_F64, "f32": AWG_LOCAL_F32, "f16x3": AWG_LOCAL_F16X3}
AWG_GENEO_DENSE, AWG_GENEO_SUBSPACE = 0, 1
COARSE2 = {"ad": 0, "inex": 1, "hyb": 2}     # second-coarse-space preconditioner (awg.h)
H2 = {"nn_hyb": 0, "asp_hyb": 1, "asp_ad": 2, "as_hyb": 3}  # two-level preconditioner for A_+ (awg.h)

STATUS = {0: "AWG_OK", 1: "AWG_NOT_CONVERGED", -1: "AWG_ERR_ARG", -2: "AWG_ERR_NOT_SYMMETRIC",
          -3: "AWG_ERR_PARTITION", -4: "AWG_ERR_MIN_OVERLAP", -5: "AWG_ERR_NOT_SPD", -6: "AWG_ERR_EIGEN",
          -7: "AWG_ERR_HIP", -8: "AWG_ERR_OOM", -9: "AWG_ERR_NONFINITE"}

EXPORTED = ["awg_default_options", "awg_setup", "awg_apply", "awg_pcg", "awg_stats", "awg_export",
            "awg_last_error", "awg_destroy", "awg_kernel_timing", "awg_kernel_times", "awg_pcg_graph",
            "awg_w_compaction", "awg_free_cached_memory",
            "awg_dense_gemm", "awg_dense_gemm_ex", "awg_dense_local_product_f16x3", "awg_dense_spd_inverse_f32",
            "awg_dense_potrf", "awg_dense_potrf_noalloc", "awg_dense_trsm",
            "awg_dense_low_eigs",
            "awg_mlp_create", "awg_mlp_num_params", "awg_mlp_get_params", "awg_mlp_set_params", "awg_mlp_forward",
            "awg_mlp_loss_grad", "awg_mlp_get_grads", "awg_mlp_adam_step", "awg_mlp_last_error", "awg_mlp_destroy",
            "awg_csr_spmm", "awg_autotune", "awg_tune_report", "awg_kernel_timing_filter", "awg_probe_mfma_f64"]
MLP_FEATURES = 12
NOALLOC_MAX_BATCH = 4096     # AWG_NOALLOC_MAX_BATCH (awg_dense.h)


class Options(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("zero_tol", ctypes.c_double), ("w_rtol", ctypes.c_double),
                ("w_maxit", ctypes.c_int32), ("local_prec", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("geneo_solver", ctypes.c_int32), ("eig_block", ctypes.c_int32), ("eig_maxit", ctypes.c_int32),
                ("eig_seed", ctypes.c_int32), ("eig_tol", ctypes.c_double), ("eig_init", ctypes.c_void_p),
                ("coords", ctypes.c_void_p), ("coord_dim", ctypes.c_int32), ("coarse2", ctypes.c_int32),
                ("h2", ctypes.c_int32), ("w_h2", ctypes.c_int32)]


class PCGInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("rel_res", ctypes.c_double),
                ("rel_res_true", ctypes.c_double), ("lmin_est", ctypes.c_double),
                ("lmax_est", ctypes.c_double), ("restarts", ctypes.c_int32), ("iters_first", ctypes.c_int32)]


class AWGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


_lib = None


def lib():
    """Load libawg.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    L.awg_default_options.argtypes = [ctypes.POINTER(Options)]
    L.awg_default_options.restype = None
    L.awg_setup.argtypes = [ctypes.POINTER(vp), i64, i64, vp, vp, vp, i32, vp, vp, ctypes.POINTER(Options)]
    L.awg_setup.restype = ctypes.c_int
    L.awg_apply.argtypes = [vp, vp, vp]
    L.awg_apply.restype = ctypes.c_int
    L.awg_pcg.argtypes = [vp, vp, vp, dbl, i32, ctypes.POINTER(PCGInfo)]
    L.awg_pcg.restype = ctypes.c_int
    L.awg_stats.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    L.awg_stats.restype = i64
    L.awg_export.argtypes = [vp, ctypes.c_char_p, vp, ctypes.c_size_t]
    L.awg_export.restype = i64
    L.awg_last_error.argtypes = [vp]
    L.awg_last_error.restype = ctypes.c_char_p
    L.awg_destroy.argtypes = [vp]
    L.awg_destroy.restype = None
    L.awg_pcg_graph.argtypes = [vp, i32]
    L.awg_pcg_graph.restype = ctypes.c_int
    L.awg_w_compaction.argtypes = [i32]
    L.awg_w_compaction.restype = ctypes.c_int
    L.awg_free_cached_memory.argtypes = [vp]
    L.awg_free_cached_memory.restype = ctypes.c_int
    L.awg_kernel_timing_filter.argtypes = [ctypes.c_char_p]
    L.awg_kernel_timing_filter.restype = ctypes.c_int
    L.awg_kernel_timing.argtypes = [i32]
    L.awg_kernel_timing.restype = ctypes.c_int
    L.awg_kernel_times.argtypes = [ctypes.c_char_p, ctypes.c_size_t, i32]
    L.awg_kernel_times.restype = i64
    L.awg_dense_gemm.argtypes = [i32, i32, i32, i32, i32, i32, dbl, vp, i32, i64, vp, i32, i64, dbl, vp, i32, i64,
                                 vp]
    L.awg_dense_gemm.restype = ctypes.c_int
    L.awg_dense_gemm_ex.argtypes = [i32, i32, i32, i32, i32, i32, dbl, vp, i32, i64, vp, vp, i32, i64, dbl, vp, i32,
                                    i64, i32, vp]
    L.awg_dense_gemm_ex.restype = ctypes.c_int
    L.awg_dense_local_product_f16x3.argtypes = [i32, vp, i32, vp, vp, vp, vp]
    L.awg_dense_local_product_f16x3.restype = ctypes.c_int
    L.awg_dense_spd_inverse_f32.argtypes = [i32, vp, vp, vp, vp, vp, vp]
    L.awg_dense_spd_inverse_f32.restype = ctypes.c_int
    L.awg_probe_mfma_f64.argtypes = [i32, ctypes.POINTER(ctypes.c_double), vp]
    L.awg_probe_mfma_f64.restype = ctypes.c_int
    L.awg_dense_potrf.argtypes = [i32, i32, vp, i32, i64, vp, vp]
    L.awg_dense_potrf.restype = ctypes.c_int
    L.awg_dense_potrf_noalloc.argtypes = [i32, i32, vp, i32, i64, vp, vp]
    L.awg_dense_potrf_noalloc.restype = ctypes.c_int
    L.awg_dense_trsm.argtypes = [i32, i32, i32, i32, vp, i32, i64, vp, i32, i64, vp]
    L.awg_dense_trsm.restype = ctypes.c_int
    L.awg_dense_low_eigs.argtypes = [i32, i32, vp, i32, i64, dbl, i32, vp, vp, vp, i64, vp]
    L.awg_dense_low_eigs.restype = ctypes.c_int
    L.awg_mlp_create.argtypes = [ctypes.POINTER(vp), i32, i32, i32, i32, ctypes.c_uint64]
    L.awg_mlp_create.restype = ctypes.c_int
    L.awg_mlp_num_params.argtypes = [vp]
    L.awg_mlp_num_params.restype = i64
    for nm in ("awg_mlp_get_params", "awg_mlp_set_params", "awg_mlp_get_grads"):
        getattr(L, nm).argtypes = [vp, vp, i64]
        getattr(L, nm).restype = ctypes.c_int
    L.awg_mlp_forward.argtypes = [vp, i64, vp, vp, i32, vp]
    L.awg_mlp_forward.restype = ctypes.c_int
    L.awg_mlp_loss_grad.argtypes = [vp, i64, vp, i32, vp, vp, vp, vp, dbl, ctypes.POINTER(dbl), vp]
    L.awg_mlp_loss_grad.restype = ctypes.c_int
    L.awg_mlp_adam_step.argtypes = [vp, dbl, dbl, dbl, dbl, vp]
    L.awg_mlp_adam_step.restype = ctypes.c_int
    L.awg_mlp_last_error.argtypes = [vp]
    L.awg_mlp_last_error.restype = ctypes.c_char_p
    L.awg_mlp_destroy.argtypes = [vp]
    L.awg_mlp_destroy.restype = None
    L.awg_csr_spmm.argtypes = [i32, i64, vp, vp, vp, vp, vp, i32, dbl, dbl, i32, vp]
    L.awg_csr_spmm.restype = ctypes.c_int
    L.awg_autotune.argtypes = [i32]
    L.awg_autotune.restype = ctypes.c_int
    L.awg_tune_report.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    L.awg_tune_report.restype = i64
    _lib = L
    return L


def kernel_timing(enable: bool) -> None:
    rc = lib().awg_kernel_timing(int(enable))
    if rc:
        raise AWGError(rc, "awg_kernel_timing")


def kernel_timing_filter(prefix: str = "") -> None:
    lib().awg_kernel_timing_filter(prefix.encode() if prefix else None)


def kernel_times(reset: bool = False) -> dict:
    L = lib()
    need = L.awg_kernel_times(None, 0, 0)
    if need < 0:
        raise AWGError(int(need), "awg_kernel_times")
    buf = ctypes.create_string_buffer(int(need) + 64)
    L.awg_kernel_times(buf, len(buf), int(reset))
    return json.loads(buf.value.decode())


def autotune(enable: bool) -> None:
    lib().awg_autotune(int(enable))


def tune_report() -> dict:
    L = lib()
    need = L.awg_tune_report(None, 0)
    buf = ctypes.create_string_buffer(int(need) + 64)
    L.awg_tune_report(buf, len(buf))
    return json.loads(buf.value.decode())


def csr_spmm(rowptr, col, val, X, Y, alpha=1.0, beta=0.0, variant=-1):
    """Y = alpha A X + beta Y (device tensors; X, Y row-major n x b float64)."""
    n = rowptr.numel() - 1
    rc = lib().awg_csr_spmm(n, col.numel(), rowptr.data_ptr(), col.data_ptr(), val.data_ptr(), X.data_ptr(),
                            Y.data_ptr(), X.shape[1], alpha, beta, variant, _stream())
    if rc:
        raise AWGError(rc, "awg_csr_spmm")
    return Y


def default_options() -> Options:
    o = Options()
    lib().awg_default_options(ctypes.byref(o))
    return o


class Solver:
    """AWG-PCG for one sparse SPD system on the current GPU.

    A: scipy CSR matrix (host) or a tuple (rowptr int64, col int32, val f64)
    of device tensors; subs: list of sorted index arrays or a tuple
    (sub_ptr int64, sub_idx int32) of device tensors.
    """

    def __init__(self, A, subs, tau: float = 0.1, local_prec: str = "f64", w_rtol: float = 1e-10,
                 w_maxit: int = 500, zero_tol: float = 1e-12, device: str = "cuda", geneo: str = "dense",
                 eig_block: int = 16, eig_maxit: int = 200, eig_tol: float = 1e-10, eig_seed: int = 0,
                 eig_init: "MLP | None" = None, coords=None, coarse2: str = "ad", h2: str = "nn_hyb",
                 w_h2: str = "asp_ad"):
        import torch
        L = lib()
        self._torch = torch
        self.device = torch.device(device)
        if isinstance(A, tuple):
            rowptr, col, val = A
            n = rowptr.numel() - 1
        else:
            A = A.tocsr()
            A.sort_indices()
            n = A.shape[0]
            rowptr = torch.as_tensor(A.indptr.astype(np.int64), device=self.device)
            col = torch.as_tensor(A.indices.astype(np.int32), device=self.device)
            val = torch.as_tensor(A.data.astype(np.float64), device=self.device)
        if isinstance(subs, tuple):
            sub_ptr, sub_idx = subs
            nsub = sub_ptr.numel() - 1
        else:
            sizes = np.array([len(s) for s in subs], dtype=np.int64)
            ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
            idx = np.concatenate([np.asarray(s) for s in subs]).astype(np.int32)
            sub_ptr = torch.as_tensor(ptr, device=self.device)
            sub_idx = torch.as_tensor(idx, device=self.device)
            nsub = len(subs)
        self.n = int(n)
        self.nnz = int(col.numel())
        self._keep = (rowptr, col, val, sub_ptr, sub_idx)
        opt = default_options()
        opt.tau = tau
        opt.zero_tol = zero_tol
        opt.w_rtol = w_rtol
        opt.w_maxit = w_maxit
        if local_prec not in LOCAL_PREC:
            raise ValueError("local_prec must be one of " + ", ".join(LOCAL_PREC))
        opt.local_prec = LOCAL_PREC[local_prec]
        opt.stream = torch.cuda.current_stream(self.device).cuda_stream
        if geneo not in ("dense", "subspace"):
            raise ValueError("geneo must be 'dense' or 'subspace'")
        opt.geneo_solver = AWG_GENEO_SUBSPACE if geneo == "subspace" else AWG_GENEO_DENSE
        if coarse2 not in COARSE2:
            raise ValueError("coarse2 must be one of " + ", ".join(COARSE2))
        opt.coarse2 = COARSE2[coarse2]
        if h2 not in H2:
            raise ValueError("h2 must be one of " + ", ".join(H2))
        opt.h2 = H2[h2]
        if w_h2 not in ("nn_hyb", "asp_hyb", "asp_ad"):
            raise ValueError("w_h2 must be one of nn_hyb, asp_hyb, asp_ad")
        opt.w_h2 = H2[w_h2]
        opt.eig_block = eig_block
        opt.eig_maxit = eig_maxit
        opt.eig_tol = eig_tol
        opt.eig_seed = eig_seed
        if eig_init is not None:
            opt.eig_init = eig_init._h
        if coords is not None:
            coords = torch.as_tensor(np.asarray(coords, dtype=np.float64) if not torch.is_tensor(coords) else coords,
                                     dtype=torch.float64, device=self.device).contiguous()
            if coords.dim() == 1:
                coords = coords[:, None]
            opt.coords = coords.data_ptr()
            opt.coord_dim = coords.shape[1]
            self._coords = coords
        self._opt = opt
        ctx = ctypes.c_void_p()
        rc = L.awg_setup(ctypes.byref(ctx), self.n, self.nnz, rowptr.data_ptr(), col.data_ptr(), val.data_ptr(),
                         nsub, sub_ptr.data_ptr(), sub_idx.data_ptr(), ctypes.byref(opt))
        if rc != 0:
            raise AWGError(rc, L.awg_last_error(None).decode())
        self._ctx = ctx

    def _check(self, rc):
        if rc < 0:
            raise AWGError(rc, lib().awg_last_error(self._ctx).decode())
        return rc

    def apply(self, r):
        """z = H r (device float64 vectors)."""
        torch = self._torch
        r = r.to(device=self.device, dtype=torch.float64).contiguous()
        z = torch.empty_like(r)
        self._check(lib().awg_apply(self._ctx, r.data_ptr(), z.data_ptr()))
        return z

    def pcg(self, b, tol: float = 1e-8, maxit: int = 1000, x=None):
        """Solve A x = b; returns (x, info dict)."""
        torch = self._torch
        b = b.to(device=self.device, dtype=torch.float64).contiguous()
        if x is None:
            x = torch.empty_like(b)
        info = PCGInfo()
        rc = self._check(lib().awg_pcg(self._ctx, b.data_ptr(), x.data_ptr(), tol, maxit, ctypes.byref(info)))
        d = {k: getattr(info, k) for k, _ in PCGInfo._fields_}
        d["status"] = STATUS.get(rc, rc)
        return x, d

    def use_graph(self, enable: bool) -> None:
        self._check(lib().awg_pcg_graph(self._ctx, int(enable)))

    def stats(self) -> dict:
        L = lib()
        need = L.awg_stats(self._ctx, None, 0)
        buf = ctypes.create_string_buffer(int(need) + 1)
        L.awg_stats(self._ctx, buf, len(buf))
        return json.loads(buf.value.decode())

    def export(self, name: str):
        L = lib()
        nbytes = L.awg_export(self._ctx, name.encode(), None, 0)
        self._check(nbytes)
        dt = (np.int32 if name in ("mult", "pair_count") else np.float32 if name == "mlp_features"
              else np.float64)
        out = np.empty(int(nbytes) // np.dtype(dt).itemsize, dtype=dt)
        if nbytes:
            self._check(L.awg_export(self._ctx, name.encode(), out.ctypes.data, int(nbytes)))
        return out

    def close(self):
        if getattr(self, "_ctx", None):
            lib().awg_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# batched dense building blocks (include/awg_dense.h), uniform batches of
# column-major float64 device tensors shaped (batch, cols, rows)
# ---------------------------------------------------------------------------
def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def dense_gemm(A, B, C, alpha=1.0, beta=0.0, transA=False, transB=False):
    """C_b = alpha op(A_b) op(B_b) + beta C_b; tensors are (batch, cols, rows)."""
    batch, ka, ma = A.shape
    _, nb, kb = B.shape
    m = ka if transA else ma
    k = ma if transA else ka
    n = kb if transB else nb
    rc = lib().awg_dense_gemm(batch, m, n, k, int(transA), int(transB), alpha, A.data_ptr(), ma, ka * ma,
                              B.data_ptr(), kb, nb * kb, beta, C.data_ptr(), C.shape[2], C.shape[1] * C.shape[2],
                              _stream())
    if rc:
        raise AWGError(rc, "awg_dense_gemm")
    return C


def dense_gemm_ex(A, B, C, alpha=1.0, beta=0.0, transA=False, transB=False, variant=-1, arows=None, k=None):
    """dense_gemm with a chosen launch variant; with arows (int32 tensor of
    batch x k row indices) A is one row-major matrix (rows, lda) whose rows
    arows[b] form the columns of A_b."""
    _, nb, kb = B.shape
    if arows is None:
        batch, ka, ma = A.shape
        m = ka if transA else ma
        kk = ma if transA else ka
        lda, sa, rows = ma, ka * ma, 0
    else:
        batch = B.shape[0]
        kk = arows.shape[1]
        m = lda = A.shape[1]
        sa, rows = 0, arows.data_ptr()
    n = kb if transB else nb
    rc = lib().awg_dense_gemm_ex(batch, m, n, kk, int(transA), int(transB), alpha, A.data_ptr(), lda, sa, rows,
                                 B.data_ptr(), kb, nb * kb, beta, C.data_ptr(), C.shape[2], C.shape[1] * C.shape[2],
                                 variant, _stream())
    if rc:
        raise AWGError(rc, "awg_dense_gemm_ex")
    return C


def dense_local_product_f16x3(sizes, X, P, Y):
    """Y_b = P_b^T X_b in the split-FP16 arithmetic of AWG_LOCAL_F16X3.
    sizes: batch sizes n_b; X, Y: (sum n_b) x ncols row-major float64 device
    tensors; P: the concatenated column-major n_b x n_b matrices (float64)."""
    sz = np.ascontiguousarray(np.asarray(sizes, dtype=np.int32))
    rc = lib().awg_dense_local_product_f16x3(len(sz), sz.ctypes.data, X.shape[1], X.data_ptr(), P.data_ptr(),
                                             Y.data_ptr(), _stream())
    if rc:
        raise AWGError(rc, "awg_dense_local_product_f16x3")
    return Y


def free_cached_memory() -> int:
    """Return the library's cached device blocks to the driver; the number of
    bytes freed."""
    out = ctypes.c_uint64(0)
    lib().awg_free_cached_memory(ctypes.byref(out))
    return int(out.value)


def w_compaction(enable: bool) -> None:
    """Process-wide switch of the column compaction in the W solves (on by
    default; W is the same bit for bit either way)."""
    lib().awg_w_compaction(int(enable))


def dense_spd_inverse_f32(sizes, A, Ainv):
    """FP32 Cholesky inverses of the SPD blocks in A (concatenated column-major
    n_b x n_b float64 device blocks) into Ainv; returns (info, pivot ratio)
    per block as numpy arrays (a block with info != 0 failed)."""
    sz = np.ascontiguousarray(np.asarray(sizes, dtype=np.int32))
    info = np.zeros(len(sz), dtype=np.int32)
    ratio = np.zeros(len(sz), dtype=np.float32)
    rc = lib().awg_dense_spd_inverse_f32(len(sz), sz.ctypes.data, A.data_ptr(), Ainv.data_ptr(), info.ctypes.data,
                                         ratio.ctypes.data, _stream())
    if rc not in (0, -5):
        raise AWGError(rc, "awg_dense_spd_inverse_f32")
    return info, ratio


def probe_mfma_f64(iters: int = 4000) -> float:
    """Sustained FP64 matrix-core rate of the device, TFLOP/s."""
    out = ctypes.c_double(0.0)
    rc = lib().awg_probe_mfma_f64(iters, ctypes.byref(out), _stream())
    if rc:
        raise AWGError(rc, "awg_probe_mfma_f64")
    return out.value


def dense_potrf(A):
    """In-place Cholesky of (batch, n, n) column-major blocks; returns info array."""
    batch, n, _ = A.shape
    info = np.zeros(batch, dtype=np.int32)
    rc = lib().awg_dense_potrf(batch, n, A.data_ptr(), n, n * n, info.ctypes.data, _stream())
    if rc not in (0, -5):
        raise AWGError(rc, "awg_dense_potrf")
    return info


def dense_potrf_noalloc(A):
    """dense_potrf through the entry point that allocates no device memory
    (batch <= NOALLOC_MAX_BATCH); returns the info array."""
    batch, n, _ = A.shape
    info = np.zeros(batch, dtype=np.int32)
    rc = lib().awg_dense_potrf_noalloc(batch, n, A.data_ptr(), n, n * n, info.ctypes.data, _stream())
    if rc not in (0, -5):
        raise AWGError(rc, "awg_dense_potrf_noalloc")
    return info


def dense_trsm(L, B, trans=False):
    batch, n, _ = L.shape
    nrhs = B.shape[1]
    rc = lib().awg_dense_trsm(batch, n, nrhs, int(trans), L.data_ptr(), n, n * n, B.data_ptr(), n, nrhs * n,
                              _stream())
    if rc:
        raise AWGError(rc, "awg_dense_trsm")
    return B


def dense_low_eigs(A, thr, max_k):
    """Eigenpairs below thr of (batch, n, n) symmetric blocks (A destroyed)."""
    import torch
    batch, n, _ = A.shape
    cnt = np.zeros(batch, dtype=np.int32)
    lam = torch.zeros(batch, max(max_k, 1), dtype=torch.float64, device=A.device)
    Z = torch.zeros(batch, max(max_k, 1), n, dtype=torch.float64, device=A.device)
    rc = lib().awg_dense_low_eigs(batch, n, A.data_ptr(), n, n * n, thr, max_k, cnt.ctypes.data,
                                  lam.data_ptr(), Z.data_ptr(), max(max_k, 1) * n, _stream())
    if rc not in (0, -1):
        raise AWGError(rc, "awg_dense_low_eigs")
    return cnt, lam, Z


# ---------------------------------------------------------------------------
# warm-start network (include/awg_mlp.h)
# ---------------------------------------------------------------------------
class MLP:
    """Per-dof perceptron on the GPU; FP32 parameters, FP32 training, BF16 or
    FP32 inference.  Tensors passed in are device tensors."""

    def __init__(self, in_features: int = MLP_FEATURES, width: int = 256, hidden_layers: int = 3,
                 out_channels: int = 8, seed: int = 0):
        h = ctypes.c_void_p()
        rc = lib().awg_mlp_create(ctypes.byref(h), in_features, width, hidden_layers, out_channels, seed)
        if rc:
            raise AWGError(rc, lib().awg_mlp_last_error(None).decode())
        self._h = h
        self.dims = [in_features] + [width] * hidden_layers + [out_channels]

    @property
    def num_params(self) -> int:
        return int(lib().awg_mlp_num_params(self._h))

    def _check(self, rc):
        if rc:
            raise AWGError(rc, lib().awg_mlp_last_error(self._h).decode())

    def get_params(self) -> np.ndarray:
        out = np.empty(self.num_params, dtype=np.float32)
        self._check(lib().awg_mlp_get_params(self._h, out.ctypes.data, out.size))
        return out

    def set_params(self, vec) -> None:
        vec = np.ascontiguousarray(vec, dtype=np.float32)
        self._check(lib().awg_mlp_set_params(self._h, vec.ctypes.data, vec.size))

    def get_grads(self) -> np.ndarray:
        out = np.empty(self.num_params, dtype=np.float32)
        self._check(lib().awg_mlp_get_grads(self._h, out.ctypes.data, out.size))
        return out

    def forward(self, X, bf16: bool = True):
        import torch
        X = X.to(dtype=torch.float32).contiguous()
        Y = torch.empty(X.shape[0], self.dims[-1], dtype=torch.float32, device=X.device)
        self._check(lib().awg_mlp_forward(self._h, X.shape[0], X.data_ptr(), Y.data_ptr(), int(bf16), _stream()))
        return Y

    def loss_grad(self, X, row_ptr, tgt_off, tgt_cols, T, ridge: float = 1e-4) -> float:
        """Loss over the subdomains (row_ptr int64, tgt_off int64, tgt_cols int32,
        T float32: device tensors); the gradient stays in the model."""
        loss = ctypes.c_double()
        self._check(lib().awg_mlp_loss_grad(self._h, X.shape[0], X.data_ptr(), row_ptr.numel() - 1,
                                            row_ptr.data_ptr(), tgt_off.data_ptr(), tgt_cols.data_ptr(),
                                            T.data_ptr(), ridge, ctypes.byref(loss), _stream()))
        return loss.value

    def adam_step(self, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
        self._check(lib().awg_mlp_adam_step(self._h, lr, beta1, beta2, eps, _stream()))

    def close(self):
        if getattr(self, "_h", None):
            lib().awg_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
