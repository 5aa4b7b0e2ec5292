"""Python binding of libjf.so (include/jf.h): argument marshalling only.

Every step of the fidelity computation runs in the library (host planner + HIP kernels).
PyTorch provides the device workspace and the stream.  There is no fallback: a missing library
or a missing GPU raises.

Names mirror the C ABI: jf_load_circuit, jf_plan_contraction, jf_plan_info, jf_fidelity_alg1,
jf_fidelity_alg2, jf_fidelity_batch, jf_is_equivalent, plus Python conveniences
(load_instance, plan, fidelity).
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import weakref

HERE = os.path.dirname(os.path.abspath(__file__))
# JF_LIB selects another build of the library (the sanitizer build of the host code, see build.py)
LIB_PATH = os.environ.get("JF_LIB") or os.path.join(HERE, "libjf.so")

JF_C128, JF_C64, JF_C64_BF16X6 = 0, 1, 2
DTYPES = {"c128": JF_C128, "c64": JF_C64, "bf16x6": JF_C64_BF16X6}
JF_FLAG_NO_CANCEL, JF_FLAG_NO_FUSE, JF_FLAG_NO_BATCH, JF_FLAG_GRAPH, JF_FLAG_NO_CHAIN = 1, 2, 4, 8, 16


def JF_FLAG_EFFORT(e: int) -> int:
    """Planner search effort: 2^(e+5) randomised greedy restarts per component (e = 1..15)."""
    return (int(e) & 15) << 8

STATUS = {0: "JF_OK", -1: "JF_E_ARG", -2: "JF_E_NOT_UNITARY", -3: "JF_E_NOT_TP", -4: "JF_E_QUBIT",
          -5: "JF_E_TOO_LARGE", -6: "JF_E_OOM", -7: "JF_E_HIP", -8: "JF_E_UNSUPPORTED"}

GATE_KINDS = {"h": 0, "s": 1, "sdg": 2, "t": 3, "tdg": 4, "x": 5, "y": 6, "z": 7, "sx": 8, "rz": 9,
              "rx": 10, "ry": 11, "su2": 12, "cx": 13, "cz": 14, "cs": 15, "swap": 16,
              "mat1": 17, "mat2": 18}
NOISE_KINDS = {"kraus": 0, "depolarizing": 1, "bit_flip": 2, "phase_flip": 3, "bit_phase_flip": 4,
               "amplitude_damping": 5}


class JfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class jf_gate(C.Structure):
    _fields_ = [("kind", C.c_int), ("q0", C.c_int), ("q1", C.c_int), ("theta", C.c_double * 3),
                ("mat", C.POINTER(C.c_double))]


class jf_noise(C.Structure):
    _fields_ = [("after_op", C.c_int), ("qubit", C.c_int), ("channel", C.c_int), ("p", C.c_double),
                ("n_kraus", C.c_int), ("kraus", C.POINTER(C.c_double))]


class jf_result(C.Structure):
    _fields_ = [("fj", C.c_double), ("one_minus_fj", C.c_double), ("imag_residual", C.c_double),
                ("kraus_terms", C.c_longlong), ("work_items", C.c_longlong),
                ("max_log2_intermediate", C.c_double), ("path_flops", C.c_double),
                ("path_bytes", C.c_double), ("seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class jf_plan_stats(C.Structure):
    _fields_ = [("n_steps", C.c_int), ("n_components", C.c_int), ("n_sliced_sites", C.c_int),
                ("n_open_bits", C.c_int), ("n_tensors_before_cancel", C.c_int),
                ("n_tensors_after_cancel", C.c_int), ("planner_seconds", C.c_double),
                ("empty_loops", C.c_double), ("alg", C.c_int), ("est_seconds", C.c_double),
                ("n_swaps_rewired", C.c_int), ("n_sliced_wires", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class jf_profile(C.Structure):
    _fields_ = [("launches", C.c_longlong), ("kernel_ms", C.c_double), ("bytes", C.c_double),
                ("flops", C.c_double), ("total_ms", C.c_double), ("max_launch_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class jf_step_profile(C.Structure):
    _fields_ = [("ms", C.c_double), ("flops", C.c_double), ("bytes", C.c_double), ("kS", C.c_int),
                ("kN", C.c_int), ("L", C.c_int), ("mode", C.c_int), ("variant", C.c_int), ("component", C.c_int),
                ("steps", C.c_int), ("threads", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class jf_decision(C.Structure):
    _fields_ = [("decision", C.c_int), ("fj_lower", C.c_double), ("fj_upper", C.c_double), ("margin", C.c_double),
                ("leaves_run", C.c_longlong), ("leaves_total", C.c_longlong), ("seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# jf_kernel_variant
KV_AUTO, KV_STAGED_256, KV_STAGED_512, KV_DIRECT_256, KV_DIRECT_512, KV_FMA, KV_GAUSS_256, KV_GAUSS_512 = range(8)
KV_CHAIN = 8  # profiles only: a chain of steps in one launch
KERNEL_VARIANTS = {"auto": KV_AUTO, "staged256": KV_STAGED_256, "staged512": KV_STAGED_512,
                   "direct256": KV_DIRECT_256, "direct512": KV_DIRECT_512, "fma": KV_FMA,
                   "gauss256": KV_GAUSS_256, "gauss512": KV_GAUSS_512}

EXPORTS = ["jf_load_circuit", "jf_plan_contraction", "jf_plan_info", "jf_plan_stats_get",
           "jf_fidelity_alg1", "jf_fidelity_alg2", "jf_batch_workspace", "jf_fidelity_batch",
           "jf_is_equivalent", "jf_free_circuit", "jf_free_plan", "jf_last_error", "jf_emulate_plan",
           "jf_profile_run", "jf_plan_describe", "jf_profile_steps", "jf_autotune", "jf_set_kernel_variant",
           "jf_decide_equivalence", "jf_workspace_release", "jf_fidelity_noalloc", "jf_stream_copy"]

_lib = None


def lib():
    """Load libjf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2103_11595_amd.build`")
    # torch ships its own HIP runtime under the same soname; load it first so that libjf binds to
    # that one runtime (device pointers and streams then come from the runtime libjf uses)
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, sz = C.c_void_p, C.c_size_t
    L.jf_load_circuit.argtypes = [C.c_int, C.POINTER(jf_gate), C.c_int, C.POINTER(jf_gate), C.c_int,
                                  C.POINTER(jf_noise), C.c_int, C.c_double, C.POINTER(vp)]
    L.jf_plan_contraction.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_uint, C.POINTER(vp)]
    L.jf_plan_info.argtypes = [vp, C.POINTER(sz), C.POINTER(jf_result)]
    L.jf_plan_stats_get.argtypes = [vp, C.POINTER(jf_plan_stats)]
    L.jf_fidelity_alg1.argtypes = [vp, vp, sz, vp, C.POINTER(jf_result), C.POINTER(C.c_double)]
    L.jf_fidelity_alg2.argtypes = [vp, vp, sz, vp, C.POINTER(jf_result)]
    L.jf_batch_workspace.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(sz)]
    L.jf_fidelity_batch.argtypes = [C.POINTER(vp), C.c_int, vp, sz, vp, C.POINTER(jf_result)]
    L.jf_is_equivalent.argtypes = [C.POINTER(jf_result), C.c_double]
    L.jf_is_equivalent.restype = C.c_int
    L.jf_free_circuit.argtypes = [vp]
    L.jf_free_circuit.restype = None
    L.jf_free_plan.argtypes = [vp]
    L.jf_free_plan.restype = None
    L.jf_last_error.restype = C.c_char_p
    L.jf_plan_describe.restype = C.c_longlong
    L.jf_emulate_plan.argtypes = [vp, C.POINTER(C.c_double), C.c_longlong]
    L.jf_profile_run.argtypes = [vp, vp, sz, vp, C.POINTER(jf_profile)]
    L.jf_plan_describe.argtypes = [vp, C.c_char_p, C.c_longlong]
    L.jf_profile_steps.argtypes = [vp, vp, sz, vp, C.POINTER(jf_step_profile), C.c_int, C.POINTER(C.c_int)]
    L.jf_autotune.argtypes = [vp, vp, sz, vp, C.c_int]
    L.jf_set_kernel_variant.argtypes = [vp, C.c_int]
    L.jf_decide_equivalence.argtypes = [vp, C.c_double, vp, sz, vp, C.POINTER(jf_decision)]
    L.jf_workspace_release.argtypes = [vp, sz]
    L.jf_fidelity_noalloc.argtypes = [vp, vp, C.POINTER(jf_result), C.POINTER(C.c_double)]
    L.jf_stream_copy.argtypes = [vp, vp, sz, C.c_int, vp, C.POINTER(C.c_double)]
    for name in EXPORTS:
        if name not in ("jf_is_equivalent", "jf_free_circuit", "jf_free_plan", "jf_last_error", "jf_plan_describe"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(st):
    if st != 0:
        raise JfError(st, lib().jf_last_error().decode())


# ---------------------------------------------------------------------------- handles ---

class Circuit:
    def __init__(self, ptr, n, n_sites):
        self.ptr = ptr
        self.n = n
        self.n_sites = n_sites

    def __del__(self):
        # at interpreter exit the module's globals may already be gone: then the process frees it
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.jf_free_circuit(self.ptr)
            self.ptr = None


class Plan:
    def __init__(self, ptr, alg, dtype, circuit):
        self.ptr = ptr
        self.alg = alg
        self.dtype = dtype
        self.circuit = circuit

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.jf_free_plan(self.ptr)
            self.ptr = None

    def info(self):
        ws = C.c_size_t()
        r = jf_result()
        _check(lib().jf_plan_info(self.ptr, C.byref(ws), C.byref(r)))
        d = r.as_dict()
        d["workspace_bytes"] = ws.value
        return d

    def stats(self):
        s = jf_plan_stats()
        _check(lib().jf_plan_stats_get(self.ptr, C.byref(s)))
        return s.as_dict()

    def describe(self):
        """Per-step shapes of the lowered program (list of dicts)."""
        L = lib()
        n = L.jf_plan_describe(self.ptr, None, 0)
        buf = C.create_string_buffer(int(n))
        L.jf_plan_describe(self.ptr, buf, n)
        keys = ["comp", "step", "level", "kS", "kN", "L", "rA", "rC", "tiles", "in_prec", "out_prec", "compute",
                "nvar", "flops", "bytes", "rowsA", "rowsC", "sA", "nC", "chain"]

        def conv(k, v):
            if k in ("in_prec", "out_prec", "compute"):
                return v
            if k in ("flops", "bytes"):
                return float(v)
            if k in ("rowsA", "rowsC", "sA", "nC"):
                return [] if v == "-" else [int(x) for x in v.split(",")]
            return int(v)
        return [{k: conv(k, v) for k, v in zip(keys, line.split())} for line in buf.value.decode().splitlines()]

    def emulate(self):
        """Host emulation of the lowered step program (validation aid): complex terms for Alg I,
        T/d^2 for Alg II."""
        import numpy as np
        info = self.info()
        n = 2 * info["kraus_terms"] if self.alg == 1 else 2
        buf = (C.c_double * n)()
        _check(lib().jf_emulate_plan(self.ptr, buf, n))
        a = np.frombuffer(buf, dtype=np.float64).copy()
        return a[0::2] + 1j * a[1::2]


def _gate_struct(g, keep):
    name, qs = g[0], g[1]
    params = list(g[2]) if len(g) > 2 else []
    s = jf_gate()
    if name not in GATE_KINDS:
        raise ValueError(f"unknown gate {name!r}")
    s.kind = GATE_KINDS[name]
    s.q0 = int(qs[0])
    s.q1 = int(qs[1]) if len(qs) > 1 else 0
    if name not in ("mat1", "mat2"):
        for i, v in enumerate(params[:3]):
            s.theta[i] = float(v)
    else:
        flat = [x for row in params[0] for z in row for x in (complex(z).real, complex(z).imag)] \
            if params and isinstance(params[0], (list, tuple)) else []
        arr = (C.c_double * len(flat))(*flat)
        keep.append(arr)
        s.mat = C.cast(arr, C.POINTER(C.c_double))
    return s


def jf_load_circuit(inst: dict, tol: float = 0.0) -> Circuit:
    """Marshal an instance dict (see paper_2103_11595_amd.instances) into jf_load_circuit."""
    keep = []
    gates = inst["gates"]
    G = (jf_gate * max(1, len(gates)))(*[_gate_struct(g, keep) for g in gates])
    noisy = inst.get("noisy_gates")
    NG = (jf_gate * max(1, len(noisy)))(*[_gate_struct(g, keep) for g in noisy]) if noisy else None
    sites = inst.get("noise", [])
    ns = []
    for s in sites:
        x = jf_noise()
        x.after_op = int(s["after"])
        x.qubit = int(s["qubit"])
        if "kraus" in s:
            x.channel = NOISE_KINDS["kraus"]
            flat = [v for K in s["kraus"] for row in K for z in row for v in (complex(z).real, complex(z).imag)]
            arr = (C.c_double * len(flat))(*flat)
            keep.append(arr)
            x.n_kraus = len(s["kraus"])
            x.kraus = C.cast(arr, C.POINTER(C.c_double))
        else:
            x.channel = NOISE_KINDS[s["channel"]]
            x.p = float(s["p"])
        ns.append(x)
    N = (jf_noise * max(1, len(ns)))(*ns)
    out = C.c_void_p()
    _check(lib().jf_load_circuit(int(inst["n"]), G, len(gates), NG, len(noisy) if noisy else 0,
                                 N, len(ns), float(tol), C.byref(out)))
    return Circuit(out.value, int(inst["n"]), len(ns))


def jf_plan_contraction(circ: Circuit, alg: int = 1, dtype="c128", max_log2: int = 0, flags: int = 0) -> Plan:
    dt = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    out = C.c_void_p()
    _check(lib().jf_plan_contraction(circ.ptr, int(alg), dt, int(max_log2), int(flags), C.byref(out)))
    p = Plan(out.value, int(alg), dt, circ)
    if int(alg) == 0:
        p.alg = p.stats()["alg"]  # the algorithm the planner chose
    return p


def jf_plan_info(plan: Plan) -> dict:
    return plan.info()


# ------------------------------------------------------------------------- GPU calls ---

def _torch_cuda():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("jf: no GPU visible; the fidelity entry points run only on the GPU")
    return torch


def _release_range(ptr: int, nbytes: int) -> None:
    if _lib is not None:
        _lib.jf_workspace_release(C.c_void_p(ptr), nbytes)


def workspace(nbytes: int, device=None):
    """Device workspace as a torch uint8 tensor (the caching allocator aligns to >= 512 bytes).
    When the tensor is collected, the library is told to forget the plan tables it held, so that
    its memory can serve again as anything, including another workspace at the same address."""
    torch = _torch_cuda()
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device or "cuda")
    weakref.finalize(t, _release_range, t.data_ptr(), t.numel()).atexit = False
    return t


def jf_workspace_release(ws) -> None:
    """Tell the library that a workspace tensor is about to be freed or reused for other data: the
    plans whose device tables it held upload them again on their next call."""
    _check(lib().jf_workspace_release(C.c_void_p(ws.data_ptr()), ws.numel()))


@contextlib.contextmanager
def _ws(ws, nbytes_fn):
    """The caller's workspace, or a temporary one that is released to the library before torch's
    caching allocator can hand its memory to anything else."""
    if ws is not None:
        yield ws
        return
    tmp = workspace(nbytes_fn())
    try:
        yield tmp
    finally:
        jf_workspace_release(tmp)


def _stream_ptr(stream):
    torch = _torch_cuda()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def jf_fidelity_alg1(plan: Plan, ws=None, stream=None, want_terms: bool = False) -> dict:
    import numpy as np
    info = plan.info()
    with _ws(ws, lambda: info["workspace_bytes"]) as ws:
        r = jf_result()
        terms = (C.c_double * (2 * info["kraus_terms"]))() if want_terms else None
        _check(lib().jf_fidelity_alg1(plan.ptr, C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream),
                                      C.byref(r), terms))
        d = r.as_dict()
        if want_terms:
            a = np.frombuffer(terms, dtype=np.float64).copy()
            d["terms"] = a[0::2] + 1j * a[1::2]
        return d


def jf_fidelity_alg2(plan: Plan, ws=None, stream=None) -> dict:
    info = plan.info()
    with _ws(ws, lambda: info["workspace_bytes"]) as ws:
        r = jf_result()
        _check(lib().jf_fidelity_alg2(plan.ptr, C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream), C.byref(r)))
        return r.as_dict()


JF_NOALLOC_BYTES = 128 << 20  # the library's static per-GPU scratch (include/jf.h)


def jf_fidelity_noalloc(plan: Plan, stream=None, want_terms: bool = False) -> dict:
    """The no-allocation entry point: the plan runs on the library's static device scratch (no
    workspace argument; plans whose workspace exceeds JF_NOALLOC_BYTES are rejected)."""
    import numpy as np
    r = jf_result()
    terms = (C.c_double * (2 * plan.info()["kraus_terms"]))() if want_terms else None
    _check(lib().jf_fidelity_noalloc(plan.ptr, _stream_ptr(stream), C.byref(r), terms))
    d = r.as_dict()
    if want_terms:
        a = np.frombuffer(terms, dtype=np.float64).copy()
        d["terms"] = a[0::2] + 1j * a[1::2]
    return d


def jf_stream_copy(src, dst, bytes_per_lane: int = 16, stream=None) -> float:
    """Milliseconds of the library's streaming copy of src into dst (torch device tensors of equal
    byte size): the HBM ceiling measurement."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    ms = C.c_double()
    _check(lib().jf_stream_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes, int(bytes_per_lane),
                                _stream_ptr(stream), C.byref(ms)))
    return ms.value


def jf_batch_workspace(plans) -> int:
    arr = (C.c_void_p * len(plans))(*[p.ptr for p in plans])
    out = C.c_size_t()
    _check(lib().jf_batch_workspace(arr, len(plans), C.byref(out)))
    return out.value


def jf_fidelity_batch(plans, ws=None, stream=None) -> list:
    arr = (C.c_void_p * len(plans))(*[p.ptr for p in plans])
    with _ws(ws, lambda: jf_batch_workspace(plans)) as ws:
        res = (jf_result * len(plans))()
        _check(lib().jf_fidelity_batch(arr, len(plans), C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream), res))
        return [r.as_dict() for r in res]


def jf_profile_run(plan: Plan, ws=None, stream=None) -> dict:
    with _ws(ws, lambda: plan.info()["workspace_bytes"]) as ws:
        r = jf_profile()
        _check(lib().jf_profile_run(plan.ptr, C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream), C.byref(r)))
        return r.as_dict()


def jf_profile_steps(plan: Plan, ws=None, stream=None) -> list:
    """Per-launch durations (ms) with flops, bytes, shape, arithmetic and kernel of each step."""
    with _ws(ws, lambda: plan.info()["workspace_bytes"]) as ws:
        n = C.c_int(0)
        _check(lib().jf_profile_steps(plan.ptr, C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream), None, 0,
                                      C.byref(n)))
        buf = (jf_step_profile * max(1, n.value))()
        _check(lib().jf_profile_steps(plan.ptr, C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream), buf,
                                      n.value, C.byref(n)))
        return [buf[i].as_dict() for i in range(n.value)]


def jf_autotune(plan: Plan, ws=None, stream=None, reps: int = 3) -> None:
    """Time every kernel that can run each step and keep the fastest (the workspace is clobbered)."""
    with _ws(ws, lambda: plan.info()["workspace_bytes"]) as ws:
        _check(lib().jf_autotune(plan.ptr, C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream), int(reps)))


def jf_set_kernel_variant(plan: Plan, variant) -> None:
    """Force one kernel (name from KERNEL_VARIANTS or its number) on every step it can run."""
    v = KERNEL_VARIANTS[variant] if isinstance(variant, str) else int(variant)
    _check(lib().jf_set_kernel_variant(plan.ptr, v))


def jf_decide_equivalence(plan: Plan, eps: float, ws=None, stream=None) -> dict:
    """Definition 1 with early stopping and a two-sided bound (decision 1 / 0 / -1)."""
    with _ws(ws, lambda: plan.info()["workspace_bytes"]) as ws:
        r = jf_decision()
        _check(lib().jf_decide_equivalence(plan.ptr, float(eps), C.c_void_p(ws.data_ptr()), ws.numel(),
                                           _stream_ptr(stream), C.byref(r)))
        return r.as_dict()


def jf_is_equivalent(result: dict, eps: float) -> bool:
    r = jf_result(**{k: result[k] for k, _ in jf_result._fields_})
    return bool(lib().jf_is_equivalent(C.byref(r), float(eps)))


# --------------------------------------------------------------------- conveniences ---

def plan(inst: dict, alg: int = 1, dtype="c128", max_log2: int = 0, flags: int = 0) -> Plan:
    return jf_plan_contraction(jf_load_circuit(inst), alg, dtype, max_log2, flags)


def fidelity(inst: dict, alg: int = 1, dtype="c128", want_terms: bool = False, **kw) -> dict:
    """F_J of an instance; alg = 0 lets the planner choose between Algorithms I and II."""
    p = plan(inst, alg, dtype, **kw)
    if p.stats()["alg"] == 1:
        return jf_fidelity_alg1(p, want_terms=want_terms)
    return jf_fidelity_alg2(p)
