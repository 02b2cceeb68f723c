"""The C-ABI library loads and exports every symbol include/rgsvd.h declares
(no compute calls: runs without a GPU); host-side argument validation."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rgsvd.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(rgsvd_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_interface():
    names = _declared()
    for n in ("rgsvd_plan", "rgsvd_run", "rgsvd_destroy", "rgsvd_strerror",
              "rgsvd_batch_plan", "rgsvd_batch_bind", "rgsvd_batch_run",
              "rgsvd_mlp_forward", "rgsvd_mlp_backward", "rgsvd_mlp_adam"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2404_09459_amd import rgsvd as R
    L = R.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert set(_declared()) == set(R.EXPORTS)


def _plan(**kw):
    from paper_2404_09459_amd import rgsvd as R
    d = dict(m=1000, p=800, n=300, k=20, oversample=10, q=1, seed=1, in_dtype=0)
    d.update(kw)
    desc = R.make_desc(**d)
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    rc = R.lib().rgsvd_plan(ctypes.byref(desc), ctypes.byref(h), ctypes.byref(ws))
    if rc == 0:
        R.lib().rgsvd_destroy(h)
    return rc, ws.value


def test_plan_validation_on_host():
    from paper_2404_09459_amd import rgsvd as R
    rc, ws = _plan()
    assert rc == 0 and ws > 0
    assert _plan(k=295, oversample=10)[0] == R.EINVAL          # k + p > min(m, n)
    assert _plan(p=25)[0] == R.EINVAL                          # k + p > min(p, n)
    assert _plan(k=0)[0] == R.EINVAL
    assert _plan(in_dtype=7)[0] == R.EINVAL
    assert _plan(mode="full")[0] == R.ENOTGMP                  # l1 + l2 < n
    assert _plan(n=50, k=20, oversample=10, mode="full")[0] == 0
    assert _plan(options=R.OPT_JACOBI_ROUNDS)[0] == 0
    assert _plan(options=R.OPT_JACOBI_SWEEPS)[0] == 0
    assert _plan(options=R.OPT_JACOBI_ROUNDS | R.OPT_JACOBI_SWEEPS)[0] == R.EINVAL
    assert _plan(options=R.OPT_JACOBI_SWEEPS | R.OPT_JACOBI_NOWAIT)[0] == 0
    assert _plan(options=0x8)[0] == R.EINVAL                   # unknown option bit
    assert R.lib().rgsvd_strerror(R.ENOTGMP).decode().startswith("full mode")


def test_run_rejects_bad_pointers_without_gpu():
    from paper_2404_09459_amd import rgsvd as R
    desc = R.make_desc(100, 90, 40, 5, 5, 1, 3, 0)
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    assert R.lib().rgsvd_plan(ctypes.byref(desc), ctypes.byref(h), ctypes.byref(ws)) == 0
    out = R.Out()
    # null inputs and a misaligned workspace are refused before any enqueue
    assert R.lib().rgsvd_run(h, None, 40, None, 40, None, None, ctypes.byref(out)) == R.EINVAL
    assert R.lib().rgsvd_run(h, ctypes.c_void_p(4096), 40, ctypes.c_void_p(8192), 40,
                             ctypes.c_void_p(4100), None, ctypes.byref(out)) == R.EWORKSPACE
    assert R.lib().rgsvd_run(h, ctypes.c_void_p(4096), 39, ctypes.c_void_p(8192), 40,
                             ctypes.c_void_p(4096), None, ctypes.byref(out)) == R.EINVAL
    R.lib().rgsvd_destroy(h)


def test_batch_plan_requires_one_power_count():
    """Every grouped launch of a batch serves all pairs at one step of the
    subspace iteration: pairs with different power counts are refused."""
    from paper_2404_09459_amd import rgsvd as R
    d0 = R.make_desc(400, 300, 100, 10, 5, 2, 1, R.F32, "mixed")
    d1 = R.make_desc(500, 350, 120, 12, 5, 1, 2, R.F32, "mixed")
    arr = (R.Desc * 2)(d0, d1)
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    assert R.lib().rgsvd_batch_plan(arr, 2, ctypes.byref(h), ctypes.byref(ws)) == R.EUNSUPPORTED
    d1.power_iters = 2
    arr = (R.Desc * 2)(d0, d1)
    assert R.lib().rgsvd_batch_plan(arr, 2, ctypes.byref(h), ctypes.byref(ws)) == 0
    R.lib().rgsvd_destroy(h)


def test_static_run_refuses_plans_above_the_scratch():
    """rgsvd_run_static checks the plan's workspace against the static
    scratch before touching the device."""
    from paper_2404_09459_amd import rgsvd as R
    desc = R.make_desc(20000, 15000, 5000, 100, 10, 2, 2, R.F32, "mixed")
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    assert R.lib().rgsvd_plan(ctypes.byref(desc), ctypes.byref(h), ctypes.byref(ws)) == 0
    assert ws.value > R.STATIC_SCRATCH_BYTES
    out = R.Out()
    rc = R.lib().rgsvd_run_static(h, ctypes.c_void_p(4096), 5000, ctypes.c_void_p(8192), 5000, None,
                                  ctypes.byref(out))
    assert rc == R.ETOOBIG
    assert "static scratch" in R.lib().rgsvd_strerror(R.ETOOBIG).decode()
    R.lib().rgsvd_destroy(h)
