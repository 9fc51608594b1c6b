"""awg_dense_potrf_noalloc (no device allocation, descriptors and info in the
library's static scratch array) against awg_dense_potrf, through the C ABI:
bit-identical factors and the same info on two calls in a row, the second
with a smaller batch and order (the scratch keeps the first call's contents),
including blocks that are not positive definite."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def spd_batch(rng, batch, n, bad=()):
    X = rng.standard_normal((batch, n, n))
    A = X @ np.transpose(X, (0, 2, 1)) + n * np.eye(n)
    for b, col in bad:                 # break positive definiteness at column col
        A[b, col, col] = -1.0
    return A


@pytest.mark.parametrize("first,second", [((300, 96), (7, 40)), ((4096, 33), (1, 1))])
def test_noalloc_matches_allocating_entry_point(gpu_lib, first, second):
    import torch
    awg = gpu_lib
    rng = np.random.default_rng(5)
    for batch, n in (first, second):
        print(f"\n[gpu case] noalloc potrf batch={batch} n={n}", flush=True)
        bad = [(batch // 2, n // 2), (batch - 1, 0)] if batch > 2 else []
        A = spd_batch(rng, batch, n, bad)
        # column-major blocks: pass the transpose (A is symmetric anyway)
        a1 = torch.as_tensor(np.ascontiguousarray(np.transpose(A, (0, 2, 1))), device="cuda")
        a2 = a1.clone()
        i1 = awg.dense_potrf(a1)
        i2 = awg.dense_potrf_noalloc(a2)
        torch.cuda.synchronize()
        assert np.array_equal(i1, i2)
        assert (i1 != 0).sum() == len(bad)
        for b, col in bad:
            assert i1[b] != 0
        # same kernels: every stored bit agrees (NaNs of the failed blocks included)
        assert torch.equal(a1.view(torch.int64), a2.view(torch.int64))
        L1 = torch.tril(a1.transpose(1, 2))
        ok = np.flatnonzero(i1 == 0)
        if ok.size:
            Lh = L1[torch.as_tensor(ok, device="cuda")].cpu().numpy()
            Ah = A[ok]
            rec = Lh @ np.transpose(Lh, (0, 2, 1))
            assert np.max(np.abs(rec - Ah)) <= 1e-10 * np.max(np.abs(Ah))


def test_noalloc_rejects_batch_beyond_scratch(gpu_lib):
    import ctypes
    import torch
    awg = gpu_lib
    a = torch.zeros((1, 4, 4), dtype=torch.float64, device="cuda")
    rc = awg.lib().awg_dense_potrf_noalloc(awg.NOALLOC_MAX_BATCH + 1, 4, a.data_ptr(), 4, 0, None, None)
    assert rc == -1
