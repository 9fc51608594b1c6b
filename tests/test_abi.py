"""The C-ABI library loads and exports every symbol include/awg.h declares
(no GPU needed: nothing is computed)."""
import ctypes
import os
import re

from paper_2106_10913_amd import awg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(awg_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_binding_list():
    assert declared_symbols() == sorted(awg.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = awg.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name
        assert isinstance(getattr(L, name), ctypes._CFuncPtr)


def test_default_options_and_setup_argument_errors():
    """Host-side argument checks run before any GPU work."""
    o = awg.default_options()
    assert o.tau == 0.1 and o.zero_tol == 1e-12 and o.w_rtol == 1e-10 and o.local_prec == 0
    assert o.geneo_solver == 0 and o.eig_block == 16 and o.eig_maxit == 200 and o.eig_tol == 1e-10
    L = awg.lib()
    ctx = ctypes.c_void_p()
    assert L.awg_setup(None, 1, 1, None, None, None, 1, None, None, None) == -1
    assert L.awg_setup(ctypes.byref(ctx), 0, 1, None, None, None, 1, None, None, None) == -1
    assert ctx.value is None
    assert b"invalid" in L.awg_last_error(None)
    o.tau = 1.5
    fake = ctypes.c_void_p(16)
    rc = L.awg_setup(ctypes.byref(ctx), 4, 4, fake, fake, fake, 1, fake, fake, ctypes.byref(o))
    assert rc == -1 and b"tau" in L.awg_last_error(None)
    for field, bad in [("geneo_solver", 2), ("eig_block", 0), ("eig_block", 65), ("eig_maxit", 0),
                       ("eig_tol", 0.0)]:
        o = awg.default_options()
        setattr(o, field, bad)
        assert L.awg_setup(ctypes.byref(ctx), 4, 4, fake, fake, fake, 1, fake, fake, ctypes.byref(o)) == -1, field
    assert L.awg_apply(None, None, None) == -1
    assert L.awg_stats(None, None, 0) == -1
    L.awg_destroy(None)


def test_noalloc_potrf_rejects_batches_beyond_its_scratch():
    """The entry point without device allocation checks its batch limit on the
    host, before any GPU work (no GPU needed)."""
    L = awg.lib()
    fake = ctypes.c_void_p(16)
    assert L.awg_dense_potrf_noalloc(awg.NOALLOC_MAX_BATCH + 1, 4, fake, 4, 16, None, None) == -1
    assert L.awg_dense_potrf_noalloc(0, 4, fake, 4, 16, None, None) == -1
    assert L.awg_dense_potrf_noalloc(1, 4, fake, 3, 16, None, None) == -1
    assert L.awg_dense_potrf_noalloc(1, 4, None, 4, 16, None, None) == -1
