"""The C-ABI library loads, exports every declared symbol, and rejects invalid
input before touching a device (runs without a GPU)."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_2311_02101_amd import hp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hp.LIB_PATH):
        from paper_2311_02101_amd import build
        build.build()
    return hp.load()


def declared_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"^\s*(?:hp_status|const char \*)\s*(hp_\w+)\s*\(", text, re.M)
    return names


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert set(hp.EXPORTS) <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    for s in (hp.HP_OK, hp.HP_EINVAL, hp.HP_ENOMEM, hp.HP_EDEVICE, hp.HP_EUNSUPPORTED):
        assert lib.hp_status_string(s).startswith(b"HP_")
    assert lib.hp_free(None) == hp.HP_OK


def _plan_status(lib, tables, ns, W, b, **kw):
    K = tables[0].shape[0]
    var = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    cl = np.concatenate([[0], np.cumsum([t.shape[1] for t in tables])]).astype(np.int64)
    lits = np.ascontiguousarray(np.concatenate(tables, axis=1), dtype=np.int32)
    W = np.ascontiguousarray(W, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    cnf = hp.HpCnf(kw.get("F", len(tables)), hp._ptr(var, ct.c_int64), hp._ptr(cl, ct.c_int64),
                   kw.get("K", K), hp._ptr(lits, ct.c_int32))
    rbm = hp.HpRbm(kw.get("rk", K), kw.get("L", W.shape[-1]), kw.get("T", W.shape[0]),
                   hp._ptr(W, ct.c_double), hp._ptr(b, ct.c_double))
    temps = kw.get("temps")
    tp = hp._ptr(np.asarray(temps, np.int32), ct.c_int32) if temps is not None else None
    sr = None
    if "size" in kw:                 # size-clustered model: [(k, l, n_temps, scale)] for K = 3..
        keep = []
        sr = (hp.HpRbm * 5)()
        for i, (k, l, t, scale) in enumerate(kw["size"]):
            Wg = np.full((max(t, 1), k, max(l, 1)), scale)
            bg = np.zeros((max(t, 1), max(l, 1)))
            keep += [Wg, bg]
            sr[i] = hp.HpRbm(k, l, t, hp._ptr(Wg, ct.c_double), hp._ptr(bg, ct.c_double))
    opts = hp.HpOpts(kw.get("B", 2), tp, kw.get("prec", hp.HP_FP64), kw.get("alpha", 1e-3), 0,
                     kw.get("threads", 0), kw.get("split", 0), kw.get("kernel", 0), 0,
                     ct.cast(sr, ct.c_void_p) if sr is not None else None, kw.get("wait", 0))
    h = ct.c_void_p()
    st = lib.hp_plan(ct.byref(h), ct.byref(cnf), ct.byref(rbm), ct.byref(opts), None)
    assert not h.value            # never a partial plan
    return st, lib.hp_last_error().decode()


CASES = [
    ("K outside 1..7", dict(K=8), hp.HP_EINVAL),
    ("rbm K mismatch", dict(rk=6), hp.HP_EINVAL),
    ("L = 0", dict(L=0), hp.HP_EINVAL),
    ("L = 9", dict(L=9), hp.HP_EINVAL),
    ("no formulas", dict(F=0), hp.HP_EINVAL),
    ("zero chains", dict(B=0), hp.HP_EINVAL),
    ("alpha > 1", dict(alpha=1.5), hp.HP_EINVAL),
    ("alpha NaN", dict(alpha=float("nan")), hp.HP_EINVAL),
    ("temperature out of range", dict(temps=[0, 2]), hp.HP_EINVAL),
    ("negative temperature", dict(temps=[-1, 0]), hp.HP_EINVAL),
    ("bad thread count", dict(threads=100), hp.HP_EINVAL),
    ("unknown precision", dict(prec=7), hp.HP_EINVAL),
    ("mixed precision with the pull kernel", dict(prec=hp.HP_MIXED_BF16, kernel=hp.KERNEL["pull"]),
     hp.HP_EUNSUPPORTED),
    ("mixed precision with a split", dict(prec=hp.HP_MIXED_BF16, split=2), hp.HP_EUNSUPPORTED),
    ("split not a power of two", dict(split=3), hp.HP_EINVAL),
    ("split too large", dict(split=32), hp.HP_EINVAL),
    ("unknown kernel variant", dict(kernel=5), hp.HP_EINVAL),
    ("negative split wait limit", dict(wait=-1), hp.HP_EINVAL),
    ("size RBM with the wrong L", dict(size=[(3, 4, 2, 0.1)]), hp.HP_EINVAL),
    ("size RBM with the wrong K", dict(size=[(4, 5, 2, 0.1)]), hp.HP_EINVAL),
    ("size RBM with another n_temps", dict(size=[(3, 3, 1, 0.1)]), hp.HP_EINVAL),
    ("size RBM with a NaN weight", dict(size=[(3, 3, 2, float("nan"))]), hp.HP_EINVAL),
    ("size-clustered model in mixed precision", dict(size=[(3, 3, 2, 0.1)], prec=hp.HP_MIXED_BF16),
     hp.HP_EUNSUPPORTED),
    ("size-clustered model with the pull kernel", dict(size=[(3, 3, 2, 0.1)], kernel=hp.KERNEL["pull"]),
     hp.HP_EUNSUPPORTED),
]


@pytest.mark.parametrize("name,kw,want", CASES, ids=[c[0] for c in CASES])
def test_invalid_arguments_rejected(lib, name, kw, want):
    T = np.array([[1, -2, 3], [2, 3, -1], [3, 1, 2]], dtype=np.int32)
    W = np.zeros((2, 3, 3))
    b = np.zeros((2, 3))
    st, msg = _plan_status(lib, [T], [3], W, b, **kw)
    assert st == want and msg


def test_invalid_tables_rejected(lib):
    W, b = np.zeros((1, 3, 3)), np.zeros((1, 3))
    good = np.array([[1, -2], [2, 3], [3, 1]], dtype=np.int32)
    st, msg = _plan_status(lib, [np.array([[1, 4], [2, 3], [3, 1]], np.int32)], [3], W, b)
    assert st == hp.HP_EINVAL and "exceeds" in msg
    st, msg = _plan_status(lib, [np.array([[1, 0], [2, 0], [3, 0]], np.int32)], [3], W, b)
    assert st == hp.HP_EINVAL and "no literal" in msg
    Wn = W.copy()
    Wn[0, 1, 1] = np.nan
    st, msg = _plan_status(lib, [good], [3], Wn, b)
    assert st == hp.HP_EINVAL and "non-finite" in msg
    st, _ = _plan_status(lib, [good], [0], W, b)
    assert st == hp.HP_EINVAL
    big = np.array([[1], [2], [3]], np.int32)
    st, msg = _plan_status(lib, [big], [40000], W, b)
    assert st == hp.HP_EUNSUPPORTED


def test_run_rejects_null_plan_and_state(lib):
    assert lib.hp_run(None, None, 1, None) == hp.HP_EINVAL
    assert lib.hp_last_error()
    assert lib.hp_check(None) == hp.HP_EINVAL
    assert lib.hp_plan_query(None, None) == hp.HP_EINVAL


def test_mlp_calls_reject_missing_buffers(lib):
    """The learned initializer's calls check their buffers before launching:
    a network without its backward workspace, or a null input, is refused
    (the pointers are never dereferenced on these paths)."""
    from paper_2311_02101_amd import learned as Lr
    Lr._lib()                                        # argtypes
    fake = ct.c_void_p(0x1000)
    no_ws = Lr.HpMlp(fake, fake, fake, fake, fake, None)
    assert lib.hp_mlp_backward(ct.byref(no_ws), fake, fake, 32, fake, None) == hp.HP_EINVAL
    assert b"null" in lib.hp_last_error()
    full = Lr.HpMlp(fake, fake, fake, fake, fake, fake)
    assert lib.hp_mlp_backward(ct.byref(full), None, fake, 32, fake, None) == hp.HP_EINVAL
    assert lib.hp_mlp_backward(ct.byref(full), fake, fake, 0, fake, None) == hp.HP_EINVAL
    assert lib.hp_mlp_forward(ct.byref(full), fake, 0, fake, None) == hp.HP_EINVAL
    assert lib.hp_mlp_adam(ct.byref(full), 1e-3, 0.9, 0.999, 1e-8, 0, None) == hp.HP_EINVAL
    assert lib.hp_mlp_sync(None, None) == hp.HP_EINVAL


def test_binding_refuses_missing_library(tmp_path, monkeypatch):
    monkeypatch.setattr(hp, "LIB_PATH", str(tmp_path / "libhp.so"))
    monkeypatch.setattr(hp, "_lib", None)
    with pytest.raises(ImportError):
        hp.load()
