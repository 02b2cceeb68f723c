"""Thin ctypes binding of librgsvd.so (argument marshalling only).

Every step of the method runs in the library's HIP kernels; PyTorch supplies
device memory and the stream.  If the library is not built this module raises
instead of falling back to anything else.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "librgsvd.so")

OK, EINVAL, ENOTGMP, EHIP, ENOMEM, EWORKSPACE, ENOMODEL, EUNSUPPORTED, ETOOBIG = 0, -1, -2, -3, -4, -5, -6, -7, -8
STATIC_SCRATCH_BYTES = 64 << 20
F64, F32 = 0, 1
PREC = {"fp64": 0, "fp32": 1, "mixed": 2}
OPT_JACOBI_ROUNDS = 0x1   # block Jacobi: every sweep one launch per round
OPT_JACOBI_SWEEPS = 0x2   # block Jacobi: every sweep one launch (a barrier between rounds) when it fits
OPT_JACOBI_NOWAIT = 0x4   # tests: the one-launch sweep barrier gives up at once (sweep-limit flag)
SIZING = {"fixed": 0, "adaptive": 1, "learned": 2}
MODE = {"truncated": 0, "full": 1}
INFO_WORDS = 8
MLP_PARAMS = 6402

FLAGS = {
    0x1: "shift_y", 0x2: "shift_w", 0x4: "chol_fail", 0x8: "jacobi_m",
    0x10: "jacobi_l1", 0x20: "beta_zero", 0x40: "alpha_zero", 0x80: "nonfinite", 0x100: "fallback",
}


class RgsvdError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {strerror(code)} ({code})")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("p", ctypes.c_int64), ("n", ctypes.c_int64),
                ("k", ctypes.c_int64), ("oversample", ctypes.c_int64),
                ("power_iters", ctypes.c_int32), ("in_dtype", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("sizing", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("options", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("tol", ctypes.c_double),
                ("block", ctypes.c_int64), ("lmax", ctypes.c_int64)]


_dp = ctypes.POINTER(ctypes.c_double)


class Out(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_void_p), ("beta", ctypes.c_void_p), ("theta", ctypes.c_void_p),
                ("P1", ctypes.c_void_p), ("P2", ctypes.c_void_p), ("D", ctypes.c_void_p),
                ("sigma_B", ctypes.c_void_p), ("U", ctypes.c_void_p), ("V", ctypes.c_void_p),
                ("R", ctypes.c_void_p), ("ldu", ctypes.c_int64), ("ldv", ctypes.c_int64),
                ("ldr", ctypes.c_int64), ("info", ctypes.c_void_p)]


class PairIO(ctypes.Structure):
    _fields_ = [("G1", ctypes.c_void_p), ("G2", ctypes.c_void_p), ("ld1", ctypes.c_int64),
                ("ld2", ctypes.c_int64), ("out", Out)]


EXPORTS = {
    # name: (restype, argtypes)
    "rgsvd_plan": (ctypes.c_int, [ctypes.POINTER(Desc), ctypes.POINTER(ctypes.c_void_p),
                                  ctypes.POINTER(ctypes.c_size_t)]),
    "rgsvd_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                 ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Out)]),
    "rgsvd_run_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                        ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(Out)]),
    "rgsvd_plan_sizes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "rgsvd_destroy": (None, [ctypes.c_void_p]),
    "rgsvd_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "rgsvd_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "rgsvd_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "rgsvd_batch_plan": (ctypes.c_int, [ctypes.POINTER(Desc), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_size_t)]),
    "rgsvd_batch_bind": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(PairIO), ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "rgsvd_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rgsvd_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Out),
                                      ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "rgsvd_batch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "rgsvd_mlp_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rgsvd_mlp_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "rgsvd_mlp_adam": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_float, ctypes.c_void_p]),
    "rgsvd_set_sizing_model": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rgsvd_probe_features": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                            ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rgsvd_gaussian": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_void_p]),
    "rgsvd_philox_words": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64,
                                          ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_int64, ctypes.c_void_p]),
    "rgsvd_selftest_mfma": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p]),
}

_LIB = None


def lib():
    """Load librgsvd.so (raises if it is not built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is not built; run paper_2404_09459_amd.build.build()")
        L = ctypes.CDLL(LIBPATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def strerror(code):
    try:
        return lib().rgsvd_strerror(code).decode()
    except Exception:  # library not loadable: still give a message
        return f"error {code}"


def check(code, where):
    if code != OK:
        raise RgsvdError(code, where)


# ---------------------------------------------------------- torch helpers ---
def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def make_desc(m, p, n, k, oversample, q, seed, in_dtype, precision="fp64", sizing="fixed",
              mode="truncated", tol=0.0, block=0, lmax=0, options=0):
    return Desc(m=m, p=p, n=n, k=k, oversample=oversample, power_iters=q, in_dtype=in_dtype,
                precision=PREC[precision], sizing=SIZING[sizing], mode=MODE[mode], options=options,
                seed=seed, tol=tol, block=block, lmax=lmax)


class Plan:
    """A plan plus its device workspace for one pair shape."""

    def __init__(self, desc, device):
        torch = _torch()
        self.desc = desc
        h = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        check(lib().rgsvd_plan(ctypes.byref(desc), ctypes.byref(h), ctypes.byref(ws)), "rgsvd_plan")
        self.h = h
        self.ws_bytes = ws.value
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        off = (-self.ws.data_ptr()) % 256
        self.ws_ptr = ctypes.c_void_p(self.ws.data_ptr() + off)
        t = ctypes.c_int64(); l1 = ctypes.c_int64(); l2 = ctypes.c_int64()
        check(lib().rgsvd_plan_sizes(h, ctypes.byref(t), ctypes.byref(l1), ctypes.byref(l2)),
              "rgsvd_plan_sizes")
        self.t, self.l1, self.l2 = t.value, l1.value, l2.value

    def __del__(self):
        try:
            if self.h:
                lib().rgsvd_destroy(self.h)
                self.h = None
        except Exception:
            pass


def alloc_outputs(t, m, p, n, N, device, uvr=True):
    torch = _torch()
    f = dict(dtype=torch.float64, device=device)
    o = dict(alpha=torch.empty(t, **f), beta=torch.empty(t, **f), theta=torch.empty(t, **f),
             P1=torch.empty(t, **f), P2=torch.empty(t, **f), D=torch.empty(2, **f),
             sigma_B=torch.empty(N, **f), info=torch.zeros(INFO_WORDS, dtype=torch.int32, device=device))
    if uvr:
        o["Ut"] = torch.empty((t, m), **f)     # U column-major == U^T row-major
        o["Vt"] = torch.empty((t, p), **f)
        o["R"] = torch.empty((t, n), **f)
    return o


def out_struct(o, m, p, n):
    return Out(alpha=_ptr(o["alpha"]), beta=_ptr(o["beta"]), theta=_ptr(o["theta"]),
               P1=_ptr(o["P1"]), P2=_ptr(o["P2"]), D=_ptr(o["D"]), sigma_B=_ptr(o["sigma_B"]),
               U=_ptr(o.get("Ut")), V=_ptr(o.get("Vt")), R=_ptr(o.get("R")),
               ldu=m, ldv=p, ldr=n, info=_ptr(o["info"]))


def run(plan, G1, G2, o):
    """Enqueue one run of `plan` on torch's current stream; returns o."""
    m, n = G1.shape
    p = G2.shape[0]
    assert G1.stride(1) == 1 and G2.stride(1) == 1, "rows of G must be contiguous"
    out = out_struct(o, m, p, n)
    check(lib().rgsvd_run(plan.h, _ptr(G1), G1.stride(0), _ptr(G2), G2.stride(0), plan.ws_ptr,
                          _stream(G1.device), ctypes.byref(out)), "rgsvd_run")
    return o


def run_static(plan, G1, G2, o):
    """Enqueue one run of `plan` in the library's static device scratch (no
    workspace, nothing allocated by the call); returns o."""
    m, n = G1.shape
    p = G2.shape[0]
    assert G1.stride(1) == 1 and G2.stride(1) == 1, "rows of G must be contiguous"
    out = out_struct(o, m, p, n)
    check(lib().rgsvd_run_static(plan.h, _ptr(G1), G1.stride(0), _ptr(G2), G2.stride(0), _stream(G1.device),
                                 ctypes.byref(out)), "rgsvd_run_static")
    return o


def autotune(plan, G1, G2, o, reps=2):
    """Pick the streaming kernels' tile shapes for `plan` by timing on these
    inputs (outputs are written); returns ((rt, js, chunk, kernel family), ms per run)."""
    m, n = G1.shape
    p = G2.shape[0]
    out = out_struct(o, m, p, n)
    ch = (ctypes.c_int32 * 4)()
    ms = ctypes.c_float()
    check(lib().rgsvd_autotune(plan.h, _ptr(G1), G1.stride(0), _ptr(G2), G2.stride(0), plan.ws_ptr,
                               _stream(G1.device), ctypes.byref(out), reps, ch, ctypes.byref(ms)), "rgsvd_autotune")
    return (ch[0], ch[1], ch[2], ch[3]), ms.value


_PLANS = {}


def rgsvd(G1, G2, k, oversample, q, seed, precision="fp64", mode="truncated", uvr=True,
          sizing="fixed", tol=0.0, block=0, lmax=0):
    """Randomized GSVD of the device pair (G1, G2); returns a dict of device
    tensors: alpha, beta, theta, P1, P2, D, sigma_B, info and (uvr) U, V, R.

    sizing="adaptive" builds each basis by Algorithm 1 (blocks of `block`
    columns, default 100, until the residual ||(I - QQ^T) G||_F < tol, at
    most `lmax` columns); `oversample` and `q` are then unused, the widths
    reached are info[1], info[2] and sigma_B holds info[1] + info[2] values."""
    torch = _torch()
    if G1.dtype != G2.dtype or G1.dtype not in (torch.float64, torch.float32):
        raise ValueError("G1, G2 must both be float64 or float32")
    if not (G1.is_cuda and G2.is_cuda):
        raise ValueError("G1, G2 must be device tensors")
    m, n = G1.shape
    p = G2.shape[0]
    dt = F64 if G1.dtype == torch.float64 else F32
    key = (m, p, n, k, oversample, q, seed, dt, precision, mode, sizing, tol, block, lmax, G1.device.index)
    plan = _PLANS.get(key)
    if plan is None:
        plan = Plan(make_desc(m, p, n, k, oversample, q, seed, dt, precision, sizing, mode, tol, block, lmax),
                    G1.device)
        _PLANS[key] = plan
    o = alloc_outputs(plan.t, m, p, n, plan.l1 + plan.l2, G1.device, uvr)
    run(plan, G1, G2, o)
    if uvr:
        o["U"] = o["Ut"].t()
        o["V"] = o["Vt"].t()
    return o


STAGE_TAGS = ["zero", "info", "gen", "nn", "tn", "reduce", "gram", "chol", "sx", "small",
              "recover", "sign", "mgram", "bjacobi"]


def profile_read(plan, maxn=1024):
    """Per-stage (tag, ms) of the last profiled run (call after a sync)."""
    ms = (ctypes.c_float * maxn)()
    tg = (ctypes.c_int32 * maxn)()
    cnt = ctypes.c_int32()
    check(lib().rgsvd_profile_read(plan.h, maxn, ms, tg, ctypes.byref(cnt)), "rgsvd_profile_read")
    return [(STAGE_TAGS[tg[i]], float(ms[i])) for i in range(min(cnt.value, maxn))]


def decode_flags(word):
    return [name for bit, name in FLAGS.items() if word & bit]


class BatchPlan:
    """One plan for a list of uneven pairs (one Desc each), run as a captured
    graph: bind once per set of device pointers, then replay."""

    def __init__(self, descs, device):
        torch = _torch()
        self.descs = list(descs)
        arr = (Desc * len(self.descs))(*self.descs)
        h = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        check(lib().rgsvd_batch_plan(arr, len(self.descs), ctypes.byref(h), ctypes.byref(ws)),
              "rgsvd_batch_plan")
        self.h = h
        self.ws = torch.empty(ws.value + 256, dtype=torch.uint8, device=device)
        off = (-self.ws.data_ptr()) % 256
        self.ws_ptr = ctypes.c_void_p(self.ws.data_ptr() + off)
        self.device = device
        self.outs = None

    def bind(self, pairs, uvr=True):
        """pairs: list of (G1, G2) device tensors; allocates and returns the
        per-pair output dicts (filled by every run)."""
        io = (PairIO * len(pairs))()
        self.outs = []
        self.keep = []
        for i, ((G1, G2), d) in enumerate(zip(pairs, self.descs)):
            m, n = G1.shape
            p = G2.shape[0]
            assert (m, p, n) == (d.m, d.p, d.n)
            t = d.n if d.mode == MODE["full"] else d.k
            N = 2 * (d.k + d.oversample)
            o = alloc_outputs(t, m, p, n, N, self.device, uvr)
            self.outs.append(o)
            self.keep.append((G1, G2))
            io[i].G1 = _ptr(G1); io[i].G2 = _ptr(G2)
            io[i].ld1 = G1.stride(0); io[i].ld2 = G2.stride(0)
            io[i].out = out_struct(o, m, p, n)
        check(lib().rgsvd_batch_bind(self.h, io, self.ws_ptr, _stream(self.device)), "rgsvd_batch_bind")
        return self.outs

    def run(self):
        check(lib().rgsvd_batch_run(self.h, _stream(self.device)), "rgsvd_batch_run")
        return self.outs

    def autotune(self, pairs, reps=2):
        """Time the tile-shape choices on this batch, then bind (capture)."""
        io = (PairIO * len(pairs))()
        outs = self.bind(pairs)   # allocate outputs and build io once
        for i, ((G1, G2), o) in enumerate(zip(pairs, outs)):
            io[i].G1 = _ptr(G1); io[i].G2 = _ptr(G2)
            io[i].ld1 = G1.stride(0); io[i].ld2 = G2.stride(0)
            io[i].out = out_struct(o, G1.shape[0], G2.shape[0], G1.shape[1])
        ch = (ctypes.c_int32 * 4)()
        ms = ctypes.c_float()
        check(lib().rgsvd_batch_autotune(self.h, io, self.ws_ptr, _stream(self.device), reps, ch,
                                         ctypes.byref(ms)), "rgsvd_batch_autotune")
        check(lib().rgsvd_batch_bind(self.h, io, self.ws_ptr, _stream(self.device)), "rgsvd_batch_bind")
        return (ch[0], ch[1], ch[2], ch[3]), ms.value

    def __del__(self):
        try:
            if self.h:
                lib().rgsvd_destroy(self.h)
                self.h = None
        except Exception:
            pass
