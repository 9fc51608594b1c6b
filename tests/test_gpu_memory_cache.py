"""The library's device memory cache: blocks released by one solver are
reused by the next set-up (with whatever they held), returned to the driver
by awg_free_cached_memory.  Two set-ups in a row, the second on recycled
memory, must give the same iterate bit for bit as one on fresh memory."""
import numpy as np
import pytest

import awg_problems as P

pytestmark = pytest.mark.gpu


def test_recycled_memory_gives_the_same_bits(gpu_lib):
    import torch
    w = P.q1_2d(m=32, boxes=(2, 2))
    b = torch.as_tensor(w.b, device="cuda")
    print("\n[gpu case] memory cache: q1_2d 32x32, three set-ups", flush=True)
    gpu_lib.free_cached_memory()
    xs = []
    for prec in ("f64", "f64", "f32"):
        s = gpu_lib.Solver(w.A, w.subs, tau=w.tau, local_prec=prec)
        x, info = s.pcg(b, tol=w.tol)
        assert info["converged"] == 1
        xs.append(x.cpu().numpy())
        s.close()
    assert np.array_equal(xs[0], xs[1])
    freed = gpu_lib.free_cached_memory()
    assert freed > 0
    assert gpu_lib.free_cached_memory() == 0
    s = gpu_lib.Solver(w.A, w.subs, tau=w.tau, local_prec="f32")
    x, info = s.pcg(b, tol=w.tol)
    s.close()
    assert np.array_equal(x.cpu().numpy(), xs[2])
