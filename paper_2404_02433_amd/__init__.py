"""MI355X (gfx950) effective-thermal-conductivity solver: Python binding.

Thin ctypes layer over ``libetc.so`` (C ABI declared in ``include/etc.h``).
It only marshals arguments: every step of the solve runs in the library's HIP
kernels.  PyTorch supplies device memory (the plan's workspace is a torch
tensor) and the current HIP stream.  There is no CPU fallback: if the library
is missing, importing the binding's functions raises.

Entry points keep the C names: ``etc_setup``, ``etc_solve``, ``etc_keff``,
``etc_get_solution``, ``etc_residual_history``, ``etc_apply_A``,
``etc_apply_Minv``, ``etc_destroy``, ``etc_last_error``; ``solve`` chains
setup, solve and K_eff for one call.
"""

from __future__ import annotations

import ctypes
import math
import os

__all__ = [
    "EtcError", "library_path", "load_library", "etc_workspace_size", "etc_setup", "etc_solve", "etc_keff",
    "etc_get_solution", "etc_residual_history", "etc_apply_A", "etc_apply_Minv", "etc_set_kernel_timer",
    "etc_kernel_time", "etc_copy_f64", "etc_destroy", "etc_last_error", "etc_version", "Plan", "solve",
    "STATUS", "etc_grad", "keff", "etc_setup_batch", "etc_batch_results", "etc_keff_batch", "solve_batch",
    "etc_solve_static", "STATIC_SCRATCH_BYTES", "etc_setup_ensemble", "etc_workspace_size_ensemble",
    "solve_ensemble",
]

_HERE = os.path.dirname(os.path.abspath(__file__))

STATUS = {0: "ok", 1: "not_converged", -1: "invalid", -2: "nomem", -3: "hip", -4: "breakdown", -5: "state",
          -6: "unsupported"}
_PREC = {"fp64": 0, "mixed": 1}
_KREF = {"mid": 0, "one": 1, "user": 2}
_DTYPE = {"float64": 0, "float32": 1}


class EtcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"etc status {status} ({STATUS.get(status, '?')}): {msg}")
        self.status = status


class _BC(ctypes.Structure):
    _fields_ = [("p_in", ctypes.c_double), ("p_out", ctypes.c_double)]


class _Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("kref_mode", ctypes.c_int),
        ("kref_user", ctypes.c_double * 5),
        ("rtol", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("refine_every", ctypes.c_int),
        ("poll_every", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("L", ctypes.c_double * 3),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("want_grad", ctypes.c_int),
        ("precond", ctypes.c_int),
        ("autotune", ctypes.c_int),
        ("use_graph", ctypes.c_int),
        ("thomas_modes", ctypes.c_int),
        ("thomas_parts", ctypes.c_int),
    ]


class _Problem(ctypes.Structure):
    _fields_ = [
        ("kappa", ctypes.c_void_p * 3),
        ("source", ctypes.c_void_p),
        ("p_in_face", ctypes.c_void_p),
        ("p_out_face", ctypes.c_void_p),
    ]


class _Result(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("status", ctypes.c_int),
        ("relres", ctypes.c_double),
        ("kref", ctypes.c_double * 5),
        ("lambda_lo", ctypes.c_double),
        ("lambda_hi", ctypes.c_double),
    ]


_SYMBOLS = {
    "etc_options_default": (None, [ctypes.POINTER(_Options)]),
    "etc_launch_info": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int)] * 5),
    "etc_workspace_size": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(_Options), ctypes.POINTER(ctypes.c_size_t)]),
    "etc_setup": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), _BC, ctypes.c_int,
                                 ctypes.POINTER(_Options), ctypes.POINTER(ctypes.c_void_p)]),
    "etc_setup_ex": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.c_int, ctypes.POINTER(ctypes.c_int64), _BC,
                                    ctypes.c_int, ctypes.POINTER(_Options), ctypes.POINTER(ctypes.c_void_p)]),
    "etc_workspace_size_ex": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                                             ctypes.c_int, ctypes.POINTER(_Options), ctypes.POINTER(ctypes.c_size_t)]),
    "etc_setup_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                                       _BC, ctypes.c_int, ctypes.POINTER(_Options), ctypes.POINTER(ctypes.c_void_p)]),
    "etc_workspace_size_batch": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_int,
                                                ctypes.c_int, ctypes.POINTER(_Options),
                                                ctypes.POINTER(ctypes.c_size_t)]),
    "etc_batch_results": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_double)]),
    "etc_keff_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]),
    "etc_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_Result)]),
    "etc_keff": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double)]),
    "etc_get_solution": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "etc_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "etc_grad_as": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "etc_residual_history": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_int)]),
    "etc_apply_A": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "etc_apply_Minv": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_double)]),
    "etc_set_kernel_timer": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "etc_kernel_time": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]),
    "etc_copy_f64": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "etc_destroy": (None, [ctypes.c_void_p]),
    "etc_setup_ensemble": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                                          ctypes.c_int, _BC, ctypes.c_int, ctypes.POINTER(_Options),
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "etc_workspace_size_ensemble": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_int,
                                                   ctypes.c_int, ctypes.POINTER(_Options),
                                                   ctypes.POINTER(ctypes.c_size_t)]),
    "etc_solve_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), _BC,
                                        ctypes.c_int, ctypes.POINTER(_Options), ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(_Result)]),
    "etc_last_error": (ctypes.c_char_p, []),
    "etc_version": (ctypes.c_char_p, []),
}

_lib = None
STATIC_SCRATCH_BYTES = 48 << 20   # ETC_STATIC_SCRATCH_BYTES of include/etc.h


def library_path() -> str:
    return os.path.join(_HERE, "libetc.so")


def load_library():
    """Load libetc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2404_02433_amd.build_lib`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SYMBOLS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def etc_last_error() -> str:
    return load_library().etc_last_error().decode()


def etc_version() -> str:
    return load_library().etc_version().decode()


def _check(status: int, allow_not_converged: bool = False) -> int:
    if status == 0 or (allow_not_converged and status == 1):
        return status
    raise EtcError(status, etc_last_error())


def _torch():
    import torch  # device memory and streams only

    return torch


def _options(precision="fp64", rtol=1e-6, max_iter=1000, refine_every=20, poll_every=8, kref="mid",
             kref_user=None, L=None, stream=None, want_grad=False, precond="dct", use_graph=False,
             autotune=False, thomas_shape=None) -> _Options:
    lib = load_library()
    o = _Options()
    lib.etc_options_default(ctypes.byref(o))
    o.precision = _PREC[precision]
    o.kref_mode = _KREF[kref]
    if kref_user is not None:
        for i in range(5):
            o.kref_user[i] = float(kref_user[i])
    o.rtol = float(rtol)
    o.max_iter = int(max_iter)
    o.refine_every = int(refine_every)
    o.poll_every = int(poll_every)
    if L is not None:
        for d in range(3):
            o.L[d] = float(L[d])
    o.stream = stream
    o.want_grad = 1 if want_grad else 0
    o.precond = {"dct": 0, "none": 1}[precond]
    o.use_graph = 1 if use_graph else 0
    o.autotune = 1 if autotune else 0
    if thomas_shape is not None:
        o.thomas_modes, o.thomas_parts = (int(v) for v in thomas_shape)
    return o


def _dims(shape):
    if len(shape) != 3:
        raise ValueError("kappa must be a 3D array")
    return (ctypes.c_int64 * 3)(*[int(s) for s in shape])


def etc_workspace_size(shape, dtype="float64", axis=0, **opts) -> int:
    o = _options(**opts)
    out = ctypes.c_size_t(0)
    _check(load_library().etc_workspace_size(_dims(shape), _DTYPE[dtype], int(axis), ctypes.byref(o),
                                             ctypes.byref(out)))
    return int(out.value)


class Plan:
    """Owns a C plan handle, its torch workspace and the stream it runs on."""

    def __init__(self, handle, workspace, kappa_shape, axis, precision, device, stream):
        self.handle = handle
        self.workspace = workspace
        self.shape = tuple(kappa_shape)
        self.axis = axis
        self.precision = precision
        self.device = device
        self.stream = stream
        order = [axis] + [d for d in range(3) if d != axis]
        self.canonical_shape = tuple(self.shape[d] for d in order)
        self.nbatch = 1

    @property
    def storage_dtype(self):
        torch = _torch()
        return torch.float32 if self.precision == "mixed" else torch.float64

    def close(self):
        if self.handle:
            load_library().etc_destroy(self.handle)
            self.handle = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def etc_setup(kappa, axis: int = 0, p_in: float = 1.0, p_out: float = 0.0, precision: str = "fp64",
              rtol: float = 1e-6, max_iter: int = 1000, refine_every: int = 20, poll_every: int = 8,
              kref: str = "mid", kref_user=None, L=None, want_grad: bool = False, source=None,
              p_in_face=None, p_out_face=None, precond: str = "dct", use_graph: bool = False,
              autotune: bool = False, thomas_shape=None) -> Plan:
    """Preparation phase on device data (user layout, load axis ``axis``).

    ``kappa`` is one tensor (isotropic) or a sequence of three tensors, the
    conductivity along user axes 0, 1, 2 (orthotropic), float64 or float32.
    ``source`` (float64, kappa's shape), ``p_in_face`` / ``p_out_face``
    (float64 over the two transverse axes in user order) are optional.
    ``use_graph`` replays the PCG passes from a captured HIP graph;
    ``autotune`` times launch-shape candidates at setup and keeps the fastest;
    ``thomas_shape`` = (modes, partitions) fixes the tridiagonal block shape."""
    torch = _torch()
    comps = list(kappa) if isinstance(kappa, (list, tuple)) else [kappa]
    if len(comps) not in (1, 3):
        raise ValueError("kappa must be one tensor or three components")
    for c in comps:
        if not isinstance(c, torch.Tensor) or c.device.type != "cuda":
            raise ValueError("kappa must be torch tensors on a GPU device")
        if c.dtype not in (torch.float64, torch.float32) or c.dtype != comps[0].dtype:
            raise ValueError("kappa must be float64 or float32 (one dtype)")
        if tuple(c.shape) != tuple(comps[0].shape):
            raise ValueError("kappa components must share one shape")
    comps = [c.contiguous() for c in comps]
    k0 = comps[0]
    dtype = "float64" if k0.dtype == torch.float64 else "float32"
    stream = torch.cuda.current_stream(k0.device)
    o = _options(precision, rtol, max_iter, refine_every, poll_every, kref, kref_user, L, stream.cuda_stream,
                 want_grad, precond, use_graph, autotune, thomas_shape)
    n = _dims(k0.shape)
    pr = _Problem()
    keep = list(comps)
    for d in range(3):
        pr.kappa[d] = comps[d].data_ptr() if len(comps) == 3 else (k0.data_ptr() if d == 0 else None)
    order = [d for d in range(3) if d != int(axis)]
    face_shape = (k0.shape[order[0]], k0.shape[order[1]])

    def f64(x, shape, name):
        if x is None:
            return None
        if x.dtype != torch.float64 or tuple(x.shape) != tuple(shape) or x.device != k0.device:
            raise ValueError(f"{name} must be a float64 tensor of shape {tuple(shape)} on kappa's device")
        x = x.contiguous()
        keep.append(x)
        return x.data_ptr()

    pr.source = f64(source, k0.shape, "source")
    pr.p_in_face = f64(p_in_face, face_shape, "p_in_face")
    pr.p_out_face = f64(p_out_face, face_shape, "p_out_face")
    nbytes = ctypes.c_size_t(0)
    _check(load_library().etc_workspace_size_ex(ctypes.byref(pr), n, _DTYPE[dtype], int(axis), ctypes.byref(o),
                                                ctypes.byref(nbytes)))
    ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=k0.device)
    o.workspace = ws.data_ptr()
    o.workspace_bytes = int(nbytes.value)
    h = ctypes.c_void_p(0)
    _check(load_library().etc_setup_ex(ctypes.byref(pr), _DTYPE[dtype], n, _BC(float(p_in), float(p_out)),
                                       int(axis), ctypes.byref(o), ctypes.byref(h)))
    del keep
    return Plan(h, ws, k0.shape, int(axis), precision, k0.device, stream)


def etc_solve_static(kappa, axis: int = 0, p_in: float = 1.0, p_out: float = 0.0, precision: str = "fp64",
                     rtol: float = 1e-6, max_iter: int = 1000, refine_every: int = 20, poll_every: int = 8,
                     kref: str = "mid", kref_user=None, L=None, precond: str = "dct", out=None) -> dict:
    """Setup, solve and K_eff of one isotropic RVE in the library's static
    scratch array (no device allocation, by the library or here): for
    callers that cannot allocate.  ``out`` is an optional caller-owned
    float64 tensor of kappa's shape that receives the solution."""
    torch = _torch()
    if not isinstance(kappa, torch.Tensor) or kappa.device.type != "cuda" or kappa.dim() != 3:
        raise ValueError("kappa must be a 3D torch tensor on a GPU device")
    if kappa.dtype not in (torch.float64, torch.float32) or not kappa.is_contiguous():
        raise ValueError("kappa must be a contiguous float64 or float32 tensor")
    if out is not None and (out.dtype != torch.float64 or tuple(out.shape) != tuple(kappa.shape)
                            or out.device != kappa.device or not out.is_contiguous()):
        raise ValueError("out must be a contiguous float64 tensor of kappa's shape on kappa's device")
    dtype = "float64" if kappa.dtype == torch.float64 else "float32"
    stream = torch.cuda.current_stream(kappa.device)
    o = _options(precision, rtol, max_iter, refine_every, poll_every, kref, kref_user, L, stream.cuda_stream,
                 False, precond, False, False)
    k_out, k_in, res = ctypes.c_double(0.0), ctypes.c_double(0.0), _Result()
    st = load_library().etc_solve_static(kappa.data_ptr(), _DTYPE[dtype], _dims(kappa.shape),
                                         _BC(float(p_in), float(p_out)), int(axis), ctypes.byref(o),
                                         None if out is None else out.data_ptr(), ctypes.byref(k_out),
                                         ctypes.byref(k_in), ctypes.byref(res))
    _check(st, allow_not_converged=True)
    return {"keff": k_out.value, "k_in": k_in.value, "iters": res.iters, "status": STATUS[res.status],
            "relres": res.relres, "kref": list(res.kref)}


def etc_setup_batch(kappa, axis: int = 0, p_in: float = 1.0, p_out: float = 0.0, precision: str = "fp64",
                    rtol: float = 1e-6, max_iter: int = 1000, refine_every: int = 20, poll_every: int = 8,
                    kref: str = "mid", kref_user=None, L=None, want_grad: bool = False,
                    precond: str = "dct", use_graph: bool = False, autotune: bool = False,
                    thomas_shape=None) -> Plan:
    """Batch of same-size RVEs: ``kappa`` has shape (B, n0, n1, n2)."""
    torch = _torch()
    if not isinstance(kappa, torch.Tensor) or kappa.device.type != "cuda" or kappa.dim() != 4:
        raise ValueError("kappa must be a 4D torch tensor (batch, n0, n1, n2) on a GPU device")
    if kappa.dtype not in (torch.float64, torch.float32):
        raise ValueError("kappa must be float64 or float32")
    kappa = kappa.contiguous()
    dtype = "float64" if kappa.dtype == torch.float64 else "float32"
    stream = torch.cuda.current_stream(kappa.device)
    o = _options(precision, rtol, max_iter, refine_every, poll_every, kref, kref_user, L, stream.cuda_stream,
                 want_grad, precond, use_graph, autotune, thomas_shape)
    nb = int(kappa.shape[0])
    n = _dims(kappa.shape[1:])
    nbytes = ctypes.c_size_t(0)
    _check(load_library().etc_workspace_size_batch(n, nb, _DTYPE[dtype], int(axis), ctypes.byref(o),
                                                   ctypes.byref(nbytes)))
    ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=kappa.device)
    o.workspace = ws.data_ptr()
    o.workspace_bytes = int(nbytes.value)
    h = ctypes.c_void_p(0)
    _check(load_library().etc_setup_batch(kappa.data_ptr(), _DTYPE[dtype], n, nb, _BC(float(p_in), float(p_out)),
                                          int(axis), ctypes.byref(o), ctypes.byref(h)))
    plan = Plan(h, ws, kappa.shape[1:], int(axis), precision, kappa.device, stream)
    plan.nbatch = nb
    plan.shape = tuple(kappa.shape)
    plan.canonical_shape = (nb,) + plan.canonical_shape
    return plan


def etc_batch_results(plan: Plan) -> dict:
    nb = plan.nbatch
    it = (ctypes.c_int * nb)()
    stt = (ctypes.c_int * nb)()
    rr = (ctypes.c_double * nb)()
    _check(load_library().etc_batch_results(plan.handle, it, stt, rr))
    return {"iters": list(it), "status": [STATUS.get(v, v) for v in stt], "relres": list(rr)}


def etc_keff_batch(plan: Plan) -> dict:
    nb = plan.nbatch
    ko = (ctypes.c_double * nb)()
    ki = (ctypes.c_double * nb)()
    _check(load_library().etc_keff_batch(plan.handle, ko, ki))
    return {"keff": list(ko), "k_in": list(ki)}


def solve_batch(kappa, axis: int = 0, **kw) -> dict:
    """Setup + solve + per-instance K_eff for a (B, n0, n1, n2) batch."""
    plan = etc_setup_batch(kappa, axis, **kw)
    out = etc_solve(plan)
    out.update(etc_batch_results(plan))
    out.update(etc_keff_batch(plan))
    plan.close()
    return out


def etc_workspace_size_ensemble(shapes, dtype="float64", axis=0, **opts) -> int:
    o = _options(**opts)
    n = len(shapes)
    dims = (ctypes.c_int64 * (3 * n))(*[int(d) for sh in shapes for d in sh])
    out = ctypes.c_size_t(0)
    _check(load_library().etc_workspace_size_ensemble(dims, n, _DTYPE[dtype], int(axis), ctypes.byref(o),
                                                      ctypes.byref(out)))
    return int(out.value)


def etc_setup_ensemble(kappas, axis: int = 0, p_in: float = 1.0, p_out: float = 0.0, precision: str = "fp64",
                       rtol: float = 1e-6, max_iter: int = 1000, refine_every: int = 20, poll_every: int = 8,
                       kref: str = "mid", kref_user=None, L=None, want_grad: bool = False, precond: str = "dct",
                       use_graph: bool = False, autotune: bool = False) -> Plan:
    """Mixed-size ensemble: a list of 3D tensors (one dtype, one device) solved
    together, every kernel of a pass one launch for all of them.  Solutions
    and gradients come back as one flat float64 tensor, the RVEs back to back
    in input order (``plan.ensemble_shapes`` splits it)."""
    torch = _torch()
    ks = list(kappas)
    if not ks:
        raise ValueError("an ensemble needs at least one RVE")
    for k in ks:
        if not isinstance(k, torch.Tensor) or k.dim() != 3 or k.device.type != "cuda":
            raise ValueError("every RVE must be a 3D torch tensor on a GPU device")
        if k.dtype not in (torch.float64, torch.float32) or k.dtype != ks[0].dtype or k.device != ks[0].device:
            raise ValueError("every RVE must be float64 or float32, one dtype on one device")
    ks = [k.contiguous() for k in ks]
    dtype = "float64" if ks[0].dtype == torch.float64 else "float32"
    device = ks[0].device
    stream = torch.cuda.current_stream(device)
    o = _options(precision, rtol, max_iter, refine_every, poll_every, kref, kref_user, L, stream.cuda_stream,
                 want_grad, precond, use_graph, autotune)
    n = len(ks)
    dims = (ctypes.c_int64 * (3 * n))(*[int(d) for k in ks for d in k.shape])
    ptrs = (ctypes.c_void_p * n)(*[k.data_ptr() for k in ks])
    nbytes = ctypes.c_size_t(0)
    _check(load_library().etc_workspace_size_ensemble(dims, n, _DTYPE[dtype], int(axis), ctypes.byref(o),
                                                      ctypes.byref(nbytes)))
    ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=device)
    o.workspace = ws.data_ptr()
    o.workspace_bytes = int(nbytes.value)
    h = ctypes.c_void_p(0)
    _check(load_library().etc_setup_ensemble(ptrs, dims, n, _DTYPE[dtype], _BC(float(p_in), float(p_out)),
                                             int(axis), ctypes.byref(o), ctypes.byref(h)))
    total = sum(k.numel() for k in ks)
    plan = Plan(h, ws, (total, 1, 1), int(axis), precision, device, stream)
    plan.shape = (total,)
    plan.nbatch = n
    plan.ensemble_shapes = [tuple(k.shape) for k in ks]
    return plan


def _split_flat(flat, shapes):
    out, off = [], 0
    for sh in shapes:
        v = math.prod(sh)
        out.append(flat[off:off + v].view(sh))
        off += v
    return out


def _split_even(kappas, parts):
    """Indices of `parts` subsets of the RVEs with about equal voxel counts
    (largest first, each to the lightest subset so far)."""
    order = sorted(range(len(kappas)), key=lambda i: -kappas[i].numel())
    bins = [[] for _ in range(parts)]
    load = [0] * parts
    for i in order:
        b = load.index(min(load))
        bins[b].append(i)
        load[b] += kappas[i].numel()
    return [sorted(b) for b in bins if b]


def _run_concurrent(torch, parts, run, device):
    """run(part) for every part, each on a stream of its own (default
    priority) driven by a host thread; the caller's stream waits for all."""
    from concurrent.futures import ThreadPoolExecutor

    main = torch.cuda.current_stream(device)
    streams = [torch.cuda.Stream(device) for _ in parts]
    for st in streams:
        st.wait_stream(main)  # the inputs were written on the caller's stream

    def on_stream(part, stream):
        with torch.cuda.stream(stream):
            return run(part)

    with ThreadPoolExecutor(max_workers=len(parts)) as ex:
        results = list(ex.map(on_stream, parts, streams))
    for st in streams:
        main.wait_stream(st)
    return results, streams


def solve_ensemble(kappas, axis: int = 0, max_batch_voxels: int = 1 << 28, want_grad: bool = False,
                   concurrent: bool = True, mode: str = "launch", streams: int = 1, **kw) -> dict:
    """K_eff of an ensemble of RVEs of mixed sizes, results in input order.

    mode "launch" (default): ensemble plans (etc_setup_ensemble) in which
    every kernel of a pass is one launch for all their RVEs, each RVE with its
    own exit test.  ``streams`` > 1 splits the RVEs into that many plans of
    about equal voxel counts, run at the same time on streams of their own
    (the kernels of one plan then overlap those of the others).
    mode "plans": RVEs of one shape are stacked into batch plans (at most
    ``max_batch_voxels`` voxels per plan); with ``concurrent`` the plans run at
    the same time, each on a stream of its own driven by a host thread.
    With ``want_grad`` the gradients dK/dkappa are returned too (one tensor
    per RVE)."""
    torch = _torch()
    if mode == "launch":
        def run_launch(part):
            plan = etc_setup_ensemble([kappas[i] for i in part], axis, want_grad=want_grad, **kw)
            etc_solve(plan)
            res = etc_batch_results(plan)
            res.update(etc_keff_batch(plan))
            res["grad"] = _split_flat(etc_grad(plan), plan.ensemble_shapes) if want_grad else None
            plan.close()
            return res

        n = len(kappas)
        parts = _split_even(kappas, max(1, min(int(streams), n)))
        if len(parts) > 1:
            results, sts = _run_concurrent(torch, parts, run_launch, kappas[0].device)
            if want_grad:
                main = torch.cuda.current_stream(kappas[0].device)
                for res in results:
                    for g in res["grad"]:
                        g.record_stream(main)
        else:
            results = [run_launch(parts[0])]
        out = {"keff": [None] * n, "k_in": [None] * n, "iters": [None] * n, "status": [None] * n,
               "relres": [None] * n, "plans": len(parts)}
        if want_grad:
            out["grad"] = [None] * n
        for part, res in zip(parts, results):
            for j, i in enumerate(part):
                for key in ("keff", "k_in", "iters", "status", "relres"):
                    out[key][i] = res[key][j]
                if want_grad:
                    out["grad"][i] = res["grad"][j]
        return out
    if mode != "plans":
        raise ValueError("mode must be 'launch' or 'plans'")
    buckets: dict = {}
    for i, k in enumerate(kappas):
        if not isinstance(k, torch.Tensor) or k.dim() != 3 or k.device.type != "cuda":
            raise ValueError("every RVE must be a 3D torch tensor on a GPU device")
        buckets.setdefault((tuple(k.shape), k.dtype), []).append(i)
    n = len(kappas)
    out = {"keff": [None] * n, "k_in": [None] * n, "iters": [None] * n, "status": [None] * n,
           "relres": [None] * n, "plans": 0}
    if want_grad:
        out["grad"] = [None] * n
    parts = []
    for (shape, _), idx in buckets.items():
        per = max(1, int(max_batch_voxels) // max(1, math.prod(shape)))
        parts += [idx[c0:c0 + per] for c0 in range(0, len(idx), per)]
    # largest batches first, so that the small ones fill in behind them
    parts.sort(key=lambda part: -len(part) * kappas[part[0]].numel())
    device = kappas[0].device if n else None

    def run(part):
        batch = torch.stack([kappas[i] for i in part])
        plan = etc_setup_batch(batch, axis, want_grad=want_grad, **kw)
        del batch
        etc_solve(plan)
        res = etc_batch_results(plan)
        res.update(etc_keff_batch(plan))
        res["grad"] = etc_grad(plan) if want_grad else None
        plan.close()
        return res

    if concurrent and len(parts) > 1:
        results, _ = _run_concurrent(torch, parts, run, device)
        if want_grad:
            main = torch.cuda.current_stream(device)
            for res in results:
                res["grad"].record_stream(main)
    else:
        results = [run(part) for part in parts]
    for part, res in zip(parts, results):
        out["plans"] += 1
        for j, i in enumerate(part):
            for key in ("keff", "k_in", "iters", "status", "relres"):
                out[key][i] = res[key][j]
            if want_grad:
                out["grad"][i] = res["grad"][j]
    return out


def etc_solve(plan: Plan, p0=None) -> dict:
    r = _Result()
    ptr = None
    if p0 is not None:
        torch = _torch()
        if p0.dtype != torch.float64 or tuple(p0.shape) != plan.shape:
            raise ValueError("p0 must be float64 with kappa's shape")
        p0 = p0.contiguous()
        ptr = p0.data_ptr()
    st = _check(load_library().etc_solve(plan.handle, ptr, ctypes.byref(r)), allow_not_converged=True)
    return {"iters": r.iters, "status": STATUS[st], "relres": r.relres, "kref": list(r.kref),
            "lambda_lo": r.lambda_lo, "lambda_hi": r.lambda_hi}


def etc_keff(plan: Plan, energy: bool = False) -> dict:
    ko, ki, ke = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(load_library().etc_keff(plan.handle, ctypes.byref(ko), ctypes.byref(ki),
                                   ctypes.byref(ke) if energy else None))
    out = {"keff": ko.value, "k_in": ki.value}
    if energy:
        out["k_energy"] = ke.value
    return out


def etc_get_solution(plan: Plan):
    torch = _torch()
    p = torch.empty(plan.shape, dtype=torch.float64, device=plan.device)
    _check(load_library().etc_get_solution(plan.handle, p.data_ptr()))
    return p


def etc_residual_history(plan: Plan, cap: int = 100000):
    buf = (ctypes.c_double * cap)()
    n = ctypes.c_int(0)
    _check(load_library().etc_residual_history(plan.handle, buf, cap, ctypes.byref(n)))
    return [buf[i] for i in range(n.value)]


def etc_grad(plan: Plan, dtype=None):
    """dK_out/dkappa (user layout) by the adjoint method, float64 by default
    or ``dtype`` = torch.float32 (e.g. kappa's own), rounded once on the
    device (etc_grad_as)."""
    torch = _torch()
    dtype = torch.float64 if dtype is None else dtype
    if dtype not in (torch.float64, torch.float32):
        raise ValueError("dtype must be torch.float64 or torch.float32")
    g = torch.empty(plan.shape, dtype=dtype, device=plan.device)
    _check(load_library().etc_grad_as(plan.handle, g.data_ptr(), _DTYPE["float64" if dtype == torch.float64 else "float32"]))
    return g


class KeffFunction:
    """torch.autograd.Function computing K_eff(kappa) with the adjoint gradient."""

    _cls = None

    @classmethod
    def get(cls):
        if cls._cls is None:
            torch = _torch()

            class _Keff(torch.autograd.Function):
                @staticmethod
                def forward(ctx, kappa, axis, p_in, p_out, precision, rtol):
                    # The adjoint solve runs here, while the plan exists, and
                    # only the gradient (kappa's dtype) is kept for backward:
                    # the plan's workspace is freed before forward returns.
                    want = bool(ctx.needs_input_grad[0])
                    plan = etc_setup(kappa.detach(), axis, p_in, p_out, precision, rtol, want_grad=want)
                    try:
                        etc_solve(plan)
                        k = etc_keff(plan)["keff"]
                        g = etc_grad(plan, kappa.dtype) if want else None
                    finally:
                        plan.close()
                    if want:
                        ctx.save_for_backward(g)
                    return torch.tensor(k, dtype=torch.float64, device=kappa.device)

                @staticmethod
                def backward(ctx, grad_out):
                    (g,) = ctx.saved_tensors
                    return (grad_out.to(g.dtype) * g), None, None, None, None, None

            cls._cls = _Keff
        return cls._cls


def keff(kappa, axis: int = 0, p_in: float = 1.0, p_out: float = 0.0, precision: str = "fp64", rtol: float = 1e-6):
    """Differentiable K_eff(kappa): a scalar tensor whose backward is etc_grad."""
    return KeffFunction.get().apply(kappa, axis, p_in, p_out, precision, rtol)


def _canon_vec(plan: Plan, x):
    torch = _torch()
    if x.dtype != plan.storage_dtype or tuple(x.shape) != plan.canonical_shape:
        raise ValueError(f"expected a {plan.storage_dtype} tensor of canonical shape {plan.canonical_shape}")
    return x.contiguous()


def etc_apply_A(plan: Plan, x, want_dot: bool = False):
    """y = A x on canonical-layout vectors of the plan's storage dtype."""
    torch = _torch()
    x = _canon_vec(plan, x)
    y = torch.empty_like(x)
    d = ctypes.c_double(0.0)
    _check(load_library().etc_apply_A(plan.handle, x.data_ptr(), y.data_ptr(), ctypes.byref(d) if want_dot else None))
    return (y, d.value) if want_dot else y


def etc_apply_Minv(plan: Plan, r, want_dot: bool = False):
    """z = A_ref^{-1} r on canonical-layout vectors of the plan's storage dtype."""
    torch = _torch()
    r = _canon_vec(plan, r)
    z = torch.empty_like(r)
    d = ctypes.c_double(0.0)
    _check(load_library().etc_apply_Minv(plan.handle, r.data_ptr(), z.data_ptr(),
                                         ctypes.byref(d) if want_dot else None))
    return (z, d.value) if want_dot else z


def etc_set_kernel_timer(plan: Plan, kernel_id: int):
    _check(load_library().etc_set_kernel_timer(plan.handle, int(kernel_id)))


def etc_kernel_time(plan: Plan):
    ms, n = ctypes.c_double(0.0), ctypes.c_int(0)
    _check(load_library().etc_kernel_time(plan.handle, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def etc_launch_info(plan: Plan) -> dict:
    """Launch shapes of a plan (stencil plane chunk, tridiagonal blocks per
    instance and block shape: modes x partitions) and whether the autotuner
    chose them."""
    kc, tb, tu, tm, tp = (ctypes.c_int() for _ in range(5))
    _check(load_library().etc_launch_info(plan.handle, ctypes.byref(kc), ctypes.byref(tb), ctypes.byref(tu),
                                          ctypes.byref(tm), ctypes.byref(tp)))
    return {"kchunk": kc.value, "thomas_blocks": tb.value, "tuned": bool(tu.value),
            "thomas_shape": (tm.value, tp.value)}


def etc_copy_f64(src, dst):
    torch = _torch()
    stream = torch.cuda.current_stream(src.device).cuda_stream
    _check(load_library().etc_copy_f64(src.data_ptr(), dst.data_ptr(), src.numel(), stream))


def etc_destroy(plan: Plan):
    plan.close()


def solve(kappa, axis: int = 0, p_in: float = 1.0, p_out: float = 0.0, precision: str = "fp64",
          rtol: float = 1e-6, max_iter: int = 1000, energy: bool = False, return_plan: bool = False, **kw) -> dict:
    """Setup + solve + K_eff in one call; returns a dict of results."""
    plan = etc_setup(kappa, axis, p_in, p_out, precision, rtol, max_iter, **kw)
    out = etc_solve(plan)
    out.update(etc_keff(plan, energy=energy))
    if return_plan:
        out["plan"] = plan
    else:
        plan.close()
    return out
