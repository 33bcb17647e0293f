"""Far-zone MVM of the uniform-basis group-by-group IE method on MI355X.

Thin ctypes binding of ``libubf.so`` (declared in ``include/ubf.h``). The
functions carry the C names without the ``ubf_`` prefix and only marshal
arguments: every stage of the product runs in the library's HIP kernels.
PyTorch supplies device memory (tensors) and the current stream.

The library must be built (``python -m paper_2501_04684_amd.build``); the
binding raises ``RuntimeError`` when it is missing instead of falling back
to any other implementation.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

__all__ = [
    "UbfError", "FAR_ILIST", "FAR_FULL", "FP32", "SPLIT_BF16", "SPLIT_FP16", "FP16", "lib",
    "library_path",
    "declared_symbols", "plan_create", "plan_create_batch", "workspace_bytes",
    "plan_bind", "plan_capture", "plan_replay", "plan_tune", "plan_schedule",
    "plan_set_basis", "network_bytes", "plan_set_networks", "far_mvm", "far_mvm_noalloc",
    "aggregate", "translate", "disaggregate",
    "plan_info", "plan_offsets", "plan_far_pairs", "plan_operator",
    "profile_begin", "profile_end", "plan_destroy", "status_string",
    "last_error", "FarField", "gmres_workspace_bytes", "gmres_create", "gmres_start",
    "gmres_step", "gmres_poll", "gmres_finish", "gmres_destroy", "gmres_norm_estimate",
    "gmres_set_shift", "Solver",
]

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HEADER = os.path.join(ROOT, "include", "ubf.h")
# UBF_LIBRARY may name another build of the same library (the host-sanitizer
# build); it is loaded exactly like the in-tree one.
library_path = os.environ.get("UBF_LIBRARY") or os.path.join(HERE, "libubf.so")

FAR_ILIST, FAR_FULL = 0, 1
FP32, SPLIT_BF16, SPLIT_FP16, FP16 = 0, 1, 2, 3
# stage-2 kernels of the 16-bit forms (enum ubf_translate_kernel)
TRANSLATE_CHUNKS, TRANSLATE_CHUNKS_WALK, TRANSLATE_ROUNDS, TRANSLATE_ROUNDS_DOUBLE = 0, 1, 2, 3
_PRECISIONS = {"fp32": FP32, "split-bf16": SPLIT_BF16, "split-fp16": SPLIT_FP16,
               "fp16": FP16, FP32: FP32, SPLIT_BF16: SPLIT_BF16, SPLIT_FP16: SPLIT_FP16,
               FP16: FP16}
_MODES = {"ilist": FAR_ILIST, "full": FAR_FULL, FAR_ILIST: FAR_ILIST,
          FAR_FULL: FAR_FULL}
# where the translation operators come from (enum ubf_operator_source)
OPERATORS_TABLE, OPERATORS_GENERATED = 0, 1
_OPERATORS = {"table": OPERATORS_TABLE, "generated": OPERATORS_GENERATED,
              OPERATORS_TABLE: OPERATORS_TABLE, OPERATORS_GENERATED: OPERATORS_GENERATED}


class UbfError(RuntimeError):
    """A non-zero status from the library, with its thread-local message."""

    def __init__(self, status: int, func: str, message: str):
        self.status = status
        super().__init__(f"{func}: {status_string(status)} ({status}): {message}")


class _Problem(ctypes.Structure):
    _fields_ = [("n_boxes", ctypes.c_int64), ("box_ijk", ctypes.c_void_p),
                ("a", ctypes.c_double), ("k", ctypes.c_double),
                ("eta", ctypes.c_double), ("n_d", ctypes.c_int32),
                ("far_mode", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("operators", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("n_boxes", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
                ("n_offsets", ctypes.c_int32), ("n_orbits", ctypes.c_int32),
                ("n_u", ctypes.c_int32), ("n_d", ctypes.c_int32),
                ("n_chunks", ctypes.c_int64), ("table_bytes", ctypes.c_int64),
                ("translate_flops", ctypes.c_double), ("mfma", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("n_scatterers", ctypes.c_int32),
                ("translate_groups", ctypes.c_int32), ("n_items", ctypes.c_int64),
                ("translate_kernel", ctypes.c_int32), ("operators", ctypes.c_int32)]


class _GmresStatus(ctypes.Structure):
    _fields_ = [("ready", ctypes.c_int32), ("done", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("max_rel_res", ctypes.c_double)]


_lib = None
_VP, _I32, _I64, _SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
_SIGS = {
    "ubf_plan_create": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.POINTER(_VP)]),
    "ubf_plan_create_batch": (ctypes.c_int, [ctypes.POINTER(_Problem), _I32, _VP,
                                             ctypes.POINTER(_VP)]),
    "ubf_workspace_bytes": (_SZ, [_VP, _I32]),
    "ubf_plan_bind": (ctypes.c_int, [_VP, _VP, _SZ, _I32, _VP]),
    "ubf_plan_set_basis": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "ubf_network_bytes": (_SZ, [_VP, _I32]),
    "ubf_plan_set_networks": (ctypes.c_int, [_VP, _I32, _VP, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "ubf_far_mvm": (ctypes.c_int, [_VP, _VP, _VP, _I32, _VP]),
    "ubf_far_mvm_noalloc": (ctypes.c_int, [_VP, _VP, _VP, _I32, _VP]),
    "ubf_plan_capture": (ctypes.c_int, [_VP, _VP, _VP, _I32]),
    "ubf_plan_replay": (ctypes.c_int, [_VP, _VP]),
    "ubf_plan_tune": (ctypes.c_int, [_VP, _I32, _I32, _VP, _VP]),
    "ubf_plan_schedule": (ctypes.c_int, [_VP, _I32, _I32, _VP]),
    "ubf_aggregate": (ctypes.c_int, [_VP, _VP, _VP, _I32, _VP]),
    "ubf_translate": (ctypes.c_int, [_VP, _VP, _VP, _I32, _VP]),
    "ubf_disaggregate": (ctypes.c_int, [_VP, _VP, _VP, _I32, _VP]),
    "ubf_plan_info": (ctypes.c_int, [_VP, ctypes.POINTER(_Info)]),
    "ubf_plan_offsets": (ctypes.c_int, [_VP, _VP]),
    "ubf_plan_far_pairs": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "ubf_plan_operator": (ctypes.c_int, [_VP, _I32, _VP]),
    "ubf_profile_begin": (ctypes.c_int, [_VP, _I32, _I32]),
    "ubf_profile_end": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "ubf_gmres_workspace_bytes": (_SZ, [_VP, _I32, _I32]),
    "ubf_gmres_create": (ctypes.c_int, [_VP, _I32, _I32, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, _I32, _VP, _SZ,
                                        ctypes.POINTER(_VP)]),
    "ubf_gmres_start": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "ubf_gmres_step": (ctypes.c_int, [_VP, _VP]),
    "ubf_gmres_poll": (ctypes.c_int, [_VP, _I32, ctypes.POINTER(_GmresStatus), _VP]),
    "ubf_gmres_finish": (ctypes.c_int, [_VP, _VP]),
    "ubf_gmres_norm_estimate": (ctypes.c_int, [_VP, _I32, ctypes.c_uint64, _VP,
                                               ctypes.POINTER(ctypes.c_double)]),
    "ubf_gmres_set_shift": (ctypes.c_int, [_VP, ctypes.c_double, ctypes.c_double]),
    "ubf_gmres_destroy": (None, [_VP]),
    "ubf_plan_destroy": (None, [_VP]),
    "ubf_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ubf_last_error": (ctypes.c_char_p, []),
}


def lib():
    """The loaded library (loaded once); RuntimeError if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise RuntimeError(
                f"{library_path} is missing: build it with "
                "`python -m paper_2501_04684_amd.build` (no fallback exists)")
        L = ctypes.CDLL(library_path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def declared_symbols():
    """Names of the functions declared in include/ubf.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ubf_[a-z_]+)\s*\(", text)))


def status_string(status: int) -> str:
    return lib().ubf_status_string(int(status)).decode()


def last_error() -> str:
    return lib().ubf_last_error().decode()


def _check(status: int, func: str):
    if status != 0:
        raise UbfError(status, func, last_error())


def _dev_ptr(t):
    """Device address of a tensor (or None/0 for NULL)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ----------------------------------------------------------------- plans

def plan_create(boxes, a: float, k: float, n_d: int, far_mode="ilist",
                eta: float = 0.0, precision: int = FP32, operators="table"):
    """Create a plan from integer box coordinates (n, 3). Host only."""
    b = np.ascontiguousarray(np.asarray(boxes, dtype=np.int32).reshape(-1, 3))
    prob = _Problem(len(b), b.ctypes.data, float(a), float(k), float(eta),
                    int(n_d), _MODES[far_mode], _PRECISIONS[precision],
                    _OPERATORS[operators])
    out = _VP()
    _check(lib().ubf_plan_create(ctypes.byref(prob), ctypes.byref(out)),
           "ubf_plan_create")
    return out.value


def plan_create_batch(scatterers, a: float, k: float, n_d: int, far_mode="ilist",
                      eta: float = 0.0, precision: int = FP32, operators="table"):
    """One plan over several scatterers, each an (n_s, 3) array of box
    coordinates; their boxes are concatenated in the given order."""
    parts = [np.asarray(b, dtype=np.int32).reshape(-1, 3) for b in scatterers]
    b = np.ascontiguousarray(np.concatenate(parts) if parts else
                             np.zeros((0, 3), np.int32))
    ptr = np.zeros(len(parts) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(q) for q in parts])
    prob = _Problem(len(b), b.ctypes.data, float(a), float(k), float(eta),
                    int(n_d), _MODES[far_mode], _PRECISIONS[precision],
                    _OPERATORS[operators])
    out = _VP()
    _check(lib().ubf_plan_create_batch(ctypes.byref(prob), len(parts),
                                       ptr.ctypes.data, ctypes.byref(out)),
           "ubf_plan_create_batch")
    return out.value


def workspace_bytes(plan, max_nrhs: int) -> int:
    return int(lib().ubf_workspace_bytes(plan, int(max_nrhs)))


def plan_bind(plan, workspace, max_nrhs: int, stream=None):
    """Bind a device workspace (a tensor or raw address) of enough bytes."""
    nbytes = workspace.numel() * workspace.element_size() \
        if hasattr(workspace, "numel") else workspace_bytes(plan, max_nrhs)
    _check(lib().ubf_plan_bind(plan, _dev_ptr(workspace), nbytes, int(max_nrhs),
                               _stream(stream)), "ubf_plan_bind")


def plan_set_basis(plan, nb_ptr=None, S=None, T=None):
    """Set per-box S_i (and optionally T_i); all None = identity basis."""
    if nb_ptr is None:
        _check(lib().ubf_plan_set_basis(plan, None, _dev_ptr(S), _dev_ptr(T)),
               "ubf_plan_set_basis")
        return
    nb = np.ascontiguousarray(np.asarray(nb_ptr, dtype=np.int64))
    _check(lib().ubf_plan_set_basis(plan, nb.ctypes.data, _dev_ptr(S), _dev_ptr(T)),
           "ubf_plan_set_basis")


def network_bytes(plan, hidden: int) -> int:
    """Bytes of the device image for networks of ``hidden`` units (0: none)."""
    return int(lib().ubf_network_bytes(plan, int(hidden)))


def plan_set_networks(plan, hidden, W1=None, b1=None, W2=None, b2=None, image=None,
                      stream=None):
    """Per-offset networks (complex64 device tensors in plan offset order:
    W1 [n_off][hidden][N_u], b1 [n_off][hidden], W2 [n_off][N_u][hidden],
    b2 [n_off][N_u]) packed into ``image`` (a device tensor of at least
    network_bytes(plan, hidden) bytes, kept by the caller); hidden = 0
    returns stage 2 to the operator table."""
    if int(hidden) == 0:
        _check(lib().ubf_plan_set_networks(plan, 0, None, None, None, None, None, 0, None),
               "ubf_plan_set_networks")
        return
    nbytes = image.numel() * image.element_size()
    _check(lib().ubf_plan_set_networks(plan, int(hidden), _dev_ptr(W1), _dev_ptr(b1),
                                       _dev_ptr(W2), _dev_ptr(b2), _dev_ptr(image), nbytes,
                                       _stream(stream)), "ubf_plan_set_networks")


def _nrhs(x, nrhs):
    return int(nrhs if nrhs is not None else (x.shape[0] if x.dim() > 1 else 1))


def far_mvm(plan, x, y, nrhs=None, stream=None):
    _check(lib().ubf_far_mvm(plan, _dev_ptr(x), _dev_ptr(y), _nrhs(x, nrhs),
                             _stream(stream)), "ubf_far_mvm")


def far_mvm_noalloc(plan, x, y, nrhs=None, stream=None):
    _check(lib().ubf_far_mvm_noalloc(plan, _dev_ptr(x), _dev_ptr(y), _nrhs(x, nrhs),
                                     _stream(stream)), "ubf_far_mvm_noalloc")


def plan_capture(plan, x, y, nrhs=None):
    """Record y = T G S x (these tensors, this nrhs) as the plan's HIP graph."""
    _check(lib().ubf_plan_capture(plan, _dev_ptr(x), _dev_ptr(y), _nrhs(x, nrhs)),
           "ubf_plan_capture")


def plan_replay(plan, stream=None):
    """Launch the captured product on the stream (default: torch's current)."""
    _check(lib().ubf_plan_replay(plan, _stream(stream)), "ubf_plan_replay")


def plan_tune(plan, nrhs: int = 1, reps: int = 5, stream=None) -> int:
    """Autotune the stage-2 schedule; returns the chosen group count (the
    kernel is plan_info()["translate_kernel"])."""
    g = ctypes.c_int32(0)
    _check(lib().ubf_plan_tune(plan, int(nrhs), int(reps), _stream(stream),
                               ctypes.byref(g)), "ubf_plan_tune")
    return g.value


def plan_schedule(plan, kernel: int, groups: int, stream=None):
    """Set the stage-2 kernel (enum ubf_translate_kernel) and workgroups."""
    _check(lib().ubf_plan_schedule(plan, int(kernel), int(groups), _stream(stream)),
           "ubf_plan_schedule")


def aggregate(plan, x, P, nrhs=None, stream=None):
    _check(lib().ubf_aggregate(plan, _dev_ptr(x), _dev_ptr(P), _nrhs(x, nrhs),
                               _stream(stream)), "ubf_aggregate")


def translate(plan, P, E, nrhs=None, stream=None):
    _check(lib().ubf_translate(plan, _dev_ptr(P), _dev_ptr(E), _nrhs(P, nrhs),
                               _stream(stream)), "ubf_translate")


def disaggregate(plan, E, y, nrhs=None, stream=None):
    _check(lib().ubf_disaggregate(plan, _dev_ptr(E), _dev_ptr(y), _nrhs(E, nrhs),
                                  _stream(stream)), "ubf_disaggregate")


def plan_info(plan) -> dict:
    info = _Info()
    _check(lib().ubf_plan_info(plan, ctypes.byref(info)), "ubf_plan_info")
    return {name: getattr(info, name) for name, _ in _Info._fields_}


def plan_offsets(plan) -> np.ndarray:
    n = plan_info(plan)["n_offsets"]
    out = np.zeros((n, 3), dtype=np.int32)
    _check(lib().ubf_plan_offsets(plan, out.ctypes.data), "ubf_plan_offsets")
    return out


def plan_far_pairs(plan):
    """(test, src, offset_index) int32 arrays in the plan's grouped order."""
    n = plan_info(plan)["n_pairs"]
    t, s, o = (np.zeros(n, dtype=np.int32) for _ in range(3))
    _check(lib().ubf_plan_far_pairs(plan, t.ctypes.data, s.ctypes.data,
                                    o.ctypes.data), "ubf_plan_far_pairs")
    return t, s, o


def plan_operator(plan, o: int) -> np.ndarray:
    nu = plan_info(plan)["n_u"]
    out = np.zeros((nu, nu), dtype=np.complex128)
    _check(lib().ubf_plan_operator(plan, int(o), out.ctypes.data),
           "ubf_plan_operator")
    return out


def profile_begin(plan, max_calls: int, every: int = 1):
    """Start recording per-stage HIP events for one in ``every`` of the
    next products on the plan (at most ``max_calls`` recorded)."""
    _check(lib().ubf_profile_begin(plan, int(max_calls), int(every)), "ubf_profile_begin")


def profile_end(plan, max_calls: int):
    """(stage_ms[3] summed, per-call ms array) of the recorded calls."""
    stage = np.zeros(3, dtype=np.float64)
    calls = np.zeros(max(1, int(max_calls)), dtype=np.float32)
    n = ctypes.c_int32(0)
    _check(lib().ubf_profile_end(plan, stage.ctypes.data, calls.ctypes.data,
                                 ctypes.byref(n)), "ubf_profile_end")
    return stage, calls[:n.value]


def plan_destroy(plan):
    if plan:
        lib().ubf_plan_destroy(plan)


# ----------------------------------------------------------------- GMRES

def gmres_workspace_bytes(plan, nrhs: int, restart: int) -> int:
    return int(lib().ubf_gmres_workspace_bytes(plan, int(nrhs), int(restart)))


def gmres_create(plan, nrhs, restart, sigma, tol, max_steps, workspace, nbytes):
    out = _VP()
    sigma = complex(sigma)
    _check(lib().ubf_gmres_create(plan, int(nrhs), int(restart), sigma.real, sigma.imag,
                                  float(tol), int(max_steps), _dev_ptr(workspace),
                                  int(nbytes), ctypes.byref(out)), "ubf_gmres_create")
    return out.value


def gmres_start(solver, b, x, stream=None):
    _check(lib().ubf_gmres_start(solver, _dev_ptr(b), _dev_ptr(x), _stream(stream)),
           "ubf_gmres_start")


def gmres_step(solver, stream=None):
    _check(lib().ubf_gmres_step(solver, _stream(stream)), "ubf_gmres_step")


def gmres_poll(solver, nrhs: int, wait: bool = False) -> dict:
    st = _GmresStatus()
    res = np.zeros(max(1, int(nrhs)), dtype=np.float64)
    _check(lib().ubf_gmres_poll(solver, int(bool(wait)), ctypes.byref(st), res.ctypes.data),
           "ubf_gmres_poll")
    out = {name: getattr(st, name) for name, _ in _GmresStatus._fields_}
    out["rel_res"] = res[:nrhs]
    return out


def gmres_finish(solver, stream=None):
    _check(lib().ubf_gmres_finish(solver, _stream(stream)), "ubf_gmres_finish")


def gmres_norm_estimate(solver, iters: int = 3, seed: int = 0, stream=None) -> float:
    """||Z^F||_2 estimate by power iteration on the device (waits)."""
    out = ctypes.c_double(0.0)
    _check(lib().ubf_gmres_norm_estimate(solver, int(iters), int(seed), _stream(stream),
                                         ctypes.byref(out)), "ubf_gmres_norm_estimate")
    return out.value


def gmres_set_shift(solver, sigma):
    sigma = complex(sigma)
    _check(lib().ubf_gmres_set_shift(solver, sigma.real, sigma.imag), "ubf_gmres_set_shift")


def gmres_destroy(solver):
    if solver:
        lib().ubf_gmres_destroy(solver)


# ----------------------------------------------------------- convenience

class FarField:
    """A plan bound to its own device workspace, with an optional basis.

    ``FarField(boxes, a, k, n_d)(x)`` returns ``y = T G S x`` for a complex64
    CUDA tensor ``x`` of shape [nrhs, sum N_b] (or [sum N_b]).

    ``scatterers`` (a list of box arrays) replaces ``boxes`` to batch several
    independent scatterers in one plan. ``operators="generated"`` makes stage
    2 evaluate the operators itself instead of reading a table (16-bit forms).
    """

    def __init__(self, boxes, a, k, n_d, far_mode="ilist", eta=0.0,
                 max_nrhs=1, device="cuda", precision=FP32, scatterers=None,
                 operators="table"):
        import torch
        if scatterers is not None:
            self.plan = plan_create_batch(scatterers, a, k, n_d, far_mode, eta,
                                          precision, operators)
        else:
            self.plan = plan_create(boxes, a, k, n_d, far_mode, eta, precision, operators)
        self.info = plan_info(self.plan)
        self.max_nrhs = int(max_nrhs)
        nbytes = workspace_bytes(self.plan, self.max_nrhs)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        addr = self.workspace.data_ptr()
        self._ws_addr = (addr + 255) & ~255
        _check(lib().ubf_plan_bind(self.plan, self._ws_addr, nbytes,
                                   self.max_nrhs, _stream(None)), "ubf_plan_bind")
        self.nb_total = self.info["n_boxes"] * self.info["n_u"]
        self._basis = None

    @classmethod
    def from_plan(cls, plan, max_nrhs=1, device="cuda", stream=None):
        """Take ownership of an existing plan handle: allocate its workspace
        (on torch's current stream) and bind it on ``stream``."""
        import torch
        self = cls.__new__(cls)
        self.plan = plan
        self.info = plan_info(plan)
        self.max_nrhs = int(max_nrhs)
        nbytes = workspace_bytes(plan, self.max_nrhs)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        self._ws_addr = (self.workspace.data_ptr() + 255) & ~255
        _check(lib().ubf_plan_bind(plan, self._ws_addr, nbytes, self.max_nrhs,
                                   _stream(stream)), "ubf_plan_bind")
        self.nb_total = self.info["n_boxes"] * self.info["n_u"]
        self._basis = None
        return self

    def set_basis(self, nb_ptr=None, S=None, T=None):
        plan_set_basis(self.plan, nb_ptr, S, T)
        self._basis = (S, T)  # keep the device matrices alive
        self.nb_total = (int(np.asarray(nb_ptr)[-1]) if nb_ptr is not None
                         else self.info["n_boxes"] * self.info["n_u"])

    def set_networks(self, W1=None, b1=None, W2=None, b2=None):
        """Let per-offset networks (Sec. 3) stand in for the operators in
        stage 2; arguments as for ``plan_set_networks`` (numpy arrays or
        tensors, moved to the device as complex64). No arguments: back to
        the operator table."""
        import torch
        if W1 is None:
            plan_set_networks(self.plan, 0)
            self._networks = None
            return
        dev = self.workspace.device
        W1, b1, W2, b2 = (torch.as_tensor(t).to(device=dev, dtype=torch.complex64).contiguous()
                          for t in (W1, b1, W2, b2))
        n_off, hidden, n_u = W1.shape
        if (n_off != self.info["n_offsets"] or n_u != self.info["n_u"]
                or tuple(b1.shape) != (n_off, hidden) or tuple(W2.shape) != (n_off, n_u, hidden)
                or tuple(b2.shape) != (n_off, n_u)):
            raise ValueError("network shapes do not match the plan's offsets and N_u")
        nbytes = network_bytes(self.plan, hidden)
        if nbytes == 0:
            raise ValueError(f"no network kernel for N_u={n_u}, hidden={hidden}")
        image = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
        plan_set_networks(self.plan, hidden, W1, b1, W2, b2, image)
        torch.cuda.current_stream(dev).synchronize()  # the weights may go now
        self._networks = image

    def __call__(self, x, out=None, stream=None):
        import torch
        x2 = x.reshape(-1, self.nb_total)
        y = torch.empty_like(x2) if out is None else out
        far_mvm(self.plan, x2, y, x2.shape[0], stream)
        return y.reshape(x.shape) if out is None else y

    def tune(self, nrhs=None, reps=5):
        g = plan_tune(self.plan, self.max_nrhs if nrhs is None else nrhs, reps)
        self.info = plan_info(self.plan)
        return g

    def schedule(self, kernel, groups):
        plan_schedule(self.plan, kernel, groups)
        self.info = plan_info(self.plan)

    def capture(self, x, y):
        """Record y = T G S x for these two tensors; run it with replay()."""
        x2 = x.reshape(-1, self.nb_total)
        plan_capture(self.plan, x2, y, x2.shape[0])
        self._graph_io = (x, y)

    def replay(self, stream=None):
        plan_replay(self.plan, stream)

    def close(self):
        plan_destroy(self.plan)
        self.plan = None

    def __del__(self):
        try:
            if getattr(self, "plan", None):
                self.close()
        except Exception:
            pass


class Solver:
    """Restarted GMRES for (sigma I + Z^F) x = b on a :class:`FarField`.

    The Krylov workspace is a device tensor owned here; every step runs in
    the library's kernels on ``stream`` (default: torch's current stream).
    ``solve(b)`` returns ``(x, status)`` for a complex64 CUDA tensor ``b`` of
    shape [nrhs, sum N_b].
    """

    def __init__(self, field: FarField, sigma, nrhs=1, restart=30, tol=1e-4,
                 max_steps=300, stream=None):
        import torch
        self.field = field
        self.nrhs = int(nrhs)
        self.stream = stream
        nbytes = gmres_workspace_bytes(field.plan, self.nrhs, restart)
        if nbytes == 0:
            raise ValueError("nrhs and restart must be in 1..64")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8,
                                     device=field.workspace.device)
        addr = (self.workspace.data_ptr() + 255) & ~255
        self.solver = gmres_create(field.plan, self.nrhs, restart, sigma, tol, max_steps,
                                   addr, nbytes)

    def norm_estimate(self, iters=3, seed=0):
        """||Z^F||_2 estimate (power iteration on the device); abandons a
        solve in progress."""
        return gmres_norm_estimate(self.solver, iters, seed, self.stream)

    def set_shift(self, sigma):
        gmres_set_shift(self.solver, sigma)

    def start(self, b, x):
        self._io = (b, x)
        gmres_start(self.solver, b, x, self.stream)

    def step(self):
        gmres_step(self.solver, self.stream)

    def poll(self, wait=False):
        return gmres_poll(self.solver, self.nrhs, wait)

    def finish(self):
        gmres_finish(self.solver, self.stream)

    def solve(self, b, x=None, check_every=1):
        """Run to convergence (or max_steps); waits for the status every
        ``check_every`` steps."""
        import torch
        x = torch.empty_like(b) if x is None else x
        self.start(b, x)
        st = self.poll(wait=True)
        n = 0
        while not st["done"]:
            self.step()
            n += 1
            if n % check_every == 0:
                st = self.poll(wait=True)
        st = self.poll(wait=True)
        self.finish()
        return x, st

    def close(self):
        gmres_destroy(self.solver)
        self.solver = None

    def __del__(self):
        try:
            if getattr(self, "solver", None):
                self.close()
        except Exception:
            pass

