"""psim: exact PEPS amplitudes of 2D random circuits on one MI355X.

Thin ctypes binding over libpsim.so (include/psim.h).  Every step of the
contraction runs in the library's HIP kernels; this module only marshals
arguments.  PyTorch supplies device memory (the workspace) and the current
HIP stream.  There is no CPU fallback: if the library is missing the import
of any entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "libpsim.so")

PSIM_OK, PSIM_EINVAL, PSIM_ENOMEM, PSIM_EDEVICE, PSIM_EUNSUPPORTED, PSIM_EINTERNAL = 0, -1, -2, -3, -4, -5
KIND = {"H": 0, "T": 1, "SX": 2, "SY": 3, "CZ": 4, "U1": 5, "U2": 6}
PREC = {"fp64": 0, "fp32": 1, "fp32_4m": 1, "fp32_3m": 2, "bf16x3": 3}
PLAN_HOST_ONLY = 1
PLAN_SPLIT_ACC = 2
PLAN_GRAPH = 4
EXPORTED = ("psim_build", "psim_peps_info", "psim_peps_free", "psim_plan", "psim_plan_info", "psim_plan_free",
            "psim_amplitudes", "psim_contract_site", "psim_tune", "psim_profile", "psim_group", "psim_group_info",
            "psim_group_amplitudes", "psim_group_free", "psim_apply", "psim_project", "psim_double_layer",
            "psim_sample_workspace", "psim_sample", "psim_amplitudes_static",
            "psim_last_error", "psim_version")
# psim_profile classes (row scheme): 0 first site of a row and the other sites
# of the first and last rows, 1 eq. S4 (interior sites of interior rows),
# 2 last site of a row, 3 rescale
KERNEL_CLASSES = ("first_site", "interior_site", "last_site", "rescale")


class PsimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"psim status {status}: {msg}")
        self.status = status


class _Gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("cycle", ctypes.c_int32), ("q0", ctypes.c_int32),
                ("q1", ctypes.c_int32), ("m", ctypes.POINTER(ctypes.c_double))]


class PlanOpts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("flags", ctypes.c_int32), ("mem_budget_bytes", ctypes.c_uint64),
                ("max_batch", ctypes.c_int32), ("sweep", ctypes.c_int32), ("device", ctypes.c_int32),
                ("tile_cfg", ctypes.c_int32)]


class PlanStats(ctypes.Structure):
    _fields_ = [("workspace_bytes", ctypes.c_uint64), ("weights_bytes", ctypes.c_uint64),
                ("peak_tensor_elems", ctypes.c_uint64), ("cmac_per_amplitude", ctypes.c_double),
                ("n_gemm_steps", ctypes.c_int64), ("L", ctypes.c_int32), ("R", ctypes.c_int32),
                ("chi", ctypes.c_int32), ("v_chunk", ctypes.c_int32), ("sweep", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("hot_cfg", ctypes.c_int32), ("peak_bytes", ctypes.c_uint64),
                ("n_tasks", ctypes.c_int64), ("w_chunk", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelStats(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("launches", ctypes.c_int64), ("cmac", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class GroupStats(ctypes.Structure):
    _fields_ = [("n_plans", ctypes.c_int32), ("descriptor_bytes", ctypes.c_uint64),
                ("grouped_launches", ctypes.c_int64)]


_lib = None


def lib(need_torch: bool = True) -> ctypes.CDLL:
    """Load libpsim.so.  torch is imported first so that the process uses one
    HIP runtime (torch's) for both torch allocations and the library."""
    global _lib
    if _lib is not None:
        return _lib
    if need_torch:
        import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_1905_08394_amd.build` first")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
    L.psim_build.argtypes = [i32, i32, ctypes.POINTER(_Gate), sz, ctypes.POINTER(vp)]
    L.psim_peps_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                 ctypes.POINTER(i64), sz]
    L.psim_peps_free.argtypes = [vp]
    L.psim_peps_free.restype = None
    L.psim_plan.argtypes = [vp, ctypes.POINTER(PlanOpts), ctypes.POINTER(vp)]
    L.psim_plan_info.argtypes = [vp, ctypes.POINTER(PlanStats)]
    L.psim_plan_free.argtypes = [vp]
    L.psim_plan_free.restype = None
    L.psim_amplitudes.argtypes = [vp, ctypes.POINTER(ctypes.c_uint8), sz, vp, sz, vp, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]
    L.psim_amplitudes_static.argtypes = [vp, ctypes.POINTER(ctypes.c_uint8), sz, vp, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]
    L.psim_contract_site.argtypes = [i32, i64, i64, i64, i64, i64, vp, i64, ctypes.POINTER(ctypes.c_double), vp,
                                     i32, vp]
    L.psim_profile.argtypes = [vp, i32, ctypes.POINTER(KernelStats)]
    L.psim_tune.argtypes = [vp, vp, sz, vp, i32, ctypes.POINTER(ctypes.c_double)]
    L.psim_group.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp)]
    L.psim_group_info.argtypes = [vp, ctypes.POINTER(GroupStats)]
    L.psim_group_amplitudes.argtypes = [vp, ctypes.POINTER(ctypes.POINTER(ctypes.c_uint8)), ctypes.POINTER(sz),
                                        ctypes.POINTER(vp), ctypes.POINTER(sz), vp,
                                        ctypes.POINTER(ctypes.POINTER(ctypes.c_double))]
    L.psim_group_free.argtypes = [vp]
    L.psim_group_free.restype = None
    L.psim_apply.argtypes = [vp, ctypes.POINTER(_Gate), sz]
    L.psim_project.argtypes = [vp, i32, i32]
    L.psim_double_layer.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(vp)]
    L.psim_sample_workspace.argtypes = [vp, ctypes.POINTER(PlanOpts), ctypes.POINTER(u64)]
    L.psim_sample.argtypes = [vp, ctypes.POINTER(PlanOpts), ctypes.POINTER(ctypes.c_double), sz, vp, sz, vp,
                              ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_double)]
    L.psim_last_error.restype = ctypes.c_char_p
    L.psim_version.restype = ctypes.c_char_p
    for f in ("psim_build", "psim_peps_info", "psim_plan", "psim_plan_info", "psim_amplitudes", "psim_amplitudes_static",
              "psim_contract_site", "psim_profile", "psim_tune", "psim_group", "psim_group_info",
              "psim_group_amplitudes", "psim_apply", "psim_project", "psim_double_layer", "psim_sample_workspace",
              "psim_sample"):
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != PSIM_OK:
        raise PsimError(status, lib().psim_last_error().decode())


def _c_gates(circuit):
    n = len(circuit.gates)
    arr = (_Gate * max(n, 1))()
    keep = []
    for i, g in enumerate(circuit.gates):
        arr[i].kind = KIND[g.kind]
        arr[i].cycle = g.cycle
        arr[i].q0 = g.q0
        arr[i].q1 = g.q1
        if g.m is not None:
            buf = (ctypes.c_double * len(g.m))(*g.m)
            keep.append(buf)
            arr[i].m = ctypes.cast(buf, ctypes.POINTER(ctypes.c_double))
    return arr, n, keep


class Peps:
    """PEPS of a circuit after gate absorption (psim_build)."""

    def __init__(self, circuit):
        L = lib()
        arr, n, keep = _c_gates(circuit)
        h = ctypes.c_void_p()
        _check(L.psim_build(circuit.lv, circuit.lh, arr, n, ctypes.byref(h)))
        self._h = h
        self.lv, self.lh = circuit.lv, circuit.lh

    @classmethod
    def _wrap(cls, h, lv, lh):
        obj = cls.__new__(cls)
        obj._h, obj.lv, obj.lh = h, lv, lh
        return obj

    def apply(self, gates):
        """More gates (rqcgen.Gate objects, or a circuit's .gates) on this
        state (psim_apply)."""
        class _C:
            pass
        c = _C()
        c.gates = list(gates)
        arr, n, keep = _c_gates(c)
        _check(lib().psim_apply(self._h, arr, n))

    def project(self, qubit: int, value: int):
        """Record the outcome |value> of measuring qubit (psim_project; unnormalised)."""
        _check(lib().psim_project(self._h, int(qubit), int(value)))

    def double_layer(self, ops) -> "Peps":
        """Double-layer network (psim_double_layer): ops has shape (lv*lh, 2,
        2, 2) complex, ops[n, s] the operator of slice s at site n."""
        o = np.ascontiguousarray(np.asarray(ops, dtype=np.complex128))
        if o.shape != (self.lv * self.lh, 2, 2, 2):
            raise ValueError(f"ops must have shape ({self.lv * self.lh}, 2, 2, 2)")
        d = np.ascontiguousarray(o.view(np.float64).reshape(-1))
        h = ctypes.c_void_p()
        _check(lib().psim_double_layer(self._h, d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(h)))
        return Peps._wrap(h, self.lv, self.lh)

    def info(self):
        L = lib()
        nb = self.lv * (self.lh - 1) + (self.lv - 1) * self.lh
        dims = (ctypes.c_int64 * max(nb, 1))()
        lv, lh, chi = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(L.psim_peps_info(self._h, ctypes.byref(lv), ctypes.byref(lh), ctypes.byref(chi), dims, nb))
        return {"lv": lv.value, "lh": lh.value, "chi": chi.value, "bond_dims": list(dims)[:nb]}

    def close(self):
        if getattr(self, "_h", None):
            lib().psim_peps_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def expectation(peps: Peps, ops: dict, **plan_kw) -> complex:
    """<psi| prod_n ops[n] |psi> for a dict {qubit: 2x2 matrix}: the
    double-layer network with slice 0 = ops[n] (identity elsewhere), one
    contraction of bitstring 0 (psim_double_layer, psim_plan,
    psim_amplitudes; plan_kw as for Plan)."""
    n = peps.lv * peps.lh
    o = np.zeros((n, 2, 2, 2), dtype=np.complex128)
    o[:, :] = np.eye(2)
    for q, m in ops.items():
        o[q, 0] = np.asarray(m, dtype=np.complex128)
    dl = peps.double_layer(o)
    plan = Plan(dl, **plan_kw)
    try:
        return complex(plan.amplitudes(np.zeros((1, n), dtype=np.uint8))[0])
    finally:
        plan.close()
        dl.close()


def _opts(prec="fp64", mem_budget=0, max_batch=1, sweep=0, device=0, graph=False, tile_cfg=0, split_acc=False):
    flags = (PLAN_GRAPH if graph else 0) | (PLAN_SPLIT_ACC if split_acc else 0)
    return PlanOpts(PREC[prec], flags, mem_budget, max_batch, sweep, device, tile_cfg)


def sample(peps: Peps, u, stream=None, **plan_kw):
    """Sequential measurement of every qubit (psim_sample) with the uniform
    numbers u (shape (n_samples, lv*lh), in [0, 1)).  plan_kw as for Plan
    (without host_only).  Returns (bits uint8 (n_samples, lv*lh), p(bits) per
    sample)."""
    import torch
    n = peps.lv * peps.lh
    uu = np.ascontiguousarray(np.asarray(u, dtype=np.float64))
    if uu.ndim != 2 or uu.shape[1] != n:
        raise ValueError(f"u must have shape (n_samples, {n})")
    o = _opts(**plan_kw)
    need = ctypes.c_uint64()
    _check(lib().psim_sample_workspace(peps._h, ctypes.byref(o), ctypes.byref(need)))
    ws = torch.empty(max(int(need.value), 1), dtype=torch.uint8, device=f"cuda:{o.device}")
    st = stream if stream is not None else torch.cuda.current_stream(o.device).cuda_stream
    bits = np.zeros(uu.shape, dtype=np.uint8)
    prob = np.zeros(uu.shape[0])
    _check(lib().psim_sample(peps._h, ctypes.byref(o), uu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             uu.shape[0], ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(st),
                             bits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                             prob.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return bits, prob


class Plan:
    """Contraction plan with packed site matrices on the device (psim_plan)."""

    def __init__(self, peps: Peps, prec: str = "fp32", mem_budget: int = 0, max_batch: int = 1, sweep: int = 0,
                 device: int = 0, host_only: bool = False, split_acc: bool = False, graph: bool = False,
                 tile_cfg: int = 0):
        L = lib()
        flags = (PLAN_HOST_ONLY if host_only else 0) | (PLAN_SPLIT_ACC if split_acc else 0) | \
            (PLAN_GRAPH if graph else 0)
        o = PlanOpts(PREC[prec], flags, mem_budget, max_batch, sweep, device, tile_cfg)
        h = ctypes.c_void_p()
        _check(L.psim_plan(peps._h, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.device = device
        self.nq = peps.lv * peps.lh
        self._ws = None

    def stats(self) -> dict:
        s = PlanStats()
        _check(lib().psim_plan_info(self._h, ctypes.byref(s)))
        return s.as_dict()

    def workspace(self):
        import torch
        need = self.stats()["workspace_bytes"]
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def amplitudes(self, bits, stream=None, rel_err: bool = False):
        """<tau|psi> for each row of bits (uint8, shape (n, lv*lh)).  With
        rel_err=True returns (amplitudes, estimated relative errors), the
        estimates from psim_amplitudes' companion sweep (NaN for FP64)."""
        import torch
        b = np.ascontiguousarray(np.asarray(bits, dtype=np.uint8))
        if b.ndim == 1:
            b = b[None, :]
        if b.shape[1] != self.nq:
            raise ValueError(f"bitstrings must have {self.nq} entries")
        out = np.zeros(2 * b.shape[0], dtype=np.float64)
        ws = self.workspace()
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        err = np.zeros(b.shape[0], dtype=np.float64) if rel_err else None
        _check(lib().psim_amplitudes(self._h, b.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), b.shape[0],
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(st),
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     err.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if rel_err else None))
        amps = out[0::2] + 1j * out[1::2]
        return (amps, err) if rel_err else amps

    def tune(self, reps: int = 2, stream=None) -> float:
        """Pick the fastest tile candidate per interior-step shape (psim_tune)."""
        import torch
        ws = self.workspace()
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        best = ctypes.c_double()
        _check(lib().psim_tune(self._h, ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(st), reps,
                               ctypes.byref(best)))
        return best.value

    def profile_start(self):
        _check(lib().psim_profile(self._h, 1, None))

    def profile_read(self) -> dict:
        out = (KernelStats * 4)()
        _check(lib().psim_profile(self._h, 2, out))
        return {name: {"ms": out[i].ms, "launches": out[i].launches, "cmac": out[i].cmac, "bytes": out[i].bytes}
                for i, name in enumerate(KERNEL_CLASSES)}

    def profile_stop(self):
        _check(lib().psim_profile(self._h, 0, None))

    def close(self):
        if getattr(self, "_h", None):
            lib().psim_plan_free(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Group:
    """Plans run together in one interleaved sweep (psim_group): different
    circuits, lattices and depths; same-kernel FP32 site contractions of a
    step are merged into one launch.  The plans must outlive the group."""

    def __init__(self, plans):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib().psim_group(arr, len(self.plans), ctypes.byref(h)))
        self._h = h

    def stats(self) -> dict:
        s = GroupStats()
        _check(lib().psim_group_info(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in GroupStats._fields_}

    def amplitudes(self, bits_list, stream=None):
        """One bitstring array per plan (uint8, shape (n_p, lv*lh)); returns a
        list of complex128 arrays."""
        import torch
        np_ = len(self.plans)
        if len(bits_list) != np_:
            raise ValueError(f"need {np_} bitstring arrays")
        bs, outs = [], []
        for p, b in zip(self.plans, bits_list):
            b = np.ascontiguousarray(np.asarray(b, dtype=np.uint8))
            if b.ndim == 1:
                b = b[None, :]
            if b.shape[1] != p.nq:
                raise ValueError(f"bitstrings must have {p.nq} entries")
            bs.append(b)
            outs.append(np.zeros(max(2 * b.shape[0], 2), dtype=np.float64))
        wss = [p.workspace() for p in self.plans]
        PU8 = ctypes.POINTER(ctypes.c_uint8)
        PD = ctypes.POINTER(ctypes.c_double)
        c_bits = (PU8 * np_)(*[b.ctypes.data_as(PU8) for b in bs])
        c_n = (ctypes.c_size_t * np_)(*[b.shape[0] for b in bs])
        c_ws = (ctypes.c_void_p * np_)(*[w.data_ptr() for w in wss])
        c_wsb = (ctypes.c_size_t * np_)(*[w.numel() for w in wss])
        c_out = (PD * np_)(*[o.ctypes.data_as(PD) for o in outs])
        dev = self.plans[0].device
        st = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
        _check(lib().psim_group_amplitudes(self._h, c_bits, c_n, c_ws, c_wsb, ctypes.c_void_p(st), c_out))
        return [o[0:2 * b.shape[0]:2] + 1j * o[1:2 * b.shape[0]:2] for o, b in zip(outs, bs)]

    def close(self):
        if getattr(self, "_h", None):
            lib().psim_group_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def contract_site(prec: str, A, W: np.ndarray, M: int, K1: int, K2: int, N: int, batch: int = 1,
                  a_batch_stride: Optional[int] = None, transpose_out: bool = False, stream=None,
                  split_acc: bool = False, tile_cfg: int = 0):
    """One site contraction (eq. S4) through the library kernels.

    A: torch complex tensor on the GPU with batch * K1 * M * K2 elements laid out
    A[z][k1][m][k2]; W: complex (K1*K2, N).  Returns a torch tensor C[z][m][n]
    (or C[z][n][m] with transpose_out)."""
    import torch
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    assert A.dtype == dt and A.is_cuda and A.is_contiguous()
    Wd = np.ascontiguousarray(np.asarray(W, dtype=np.complex128)).view(np.float64)
    C = torch.empty(batch * M * N, dtype=dt, device=A.device)
    st = stream if stream is not None else torch.cuda.current_stream(A.device).cuda_stream
    code = PREC[prec] | (0x100 if split_acc else 0) | (tile_cfg << 16)
    _check(lib().psim_contract_site(code, batch, M, K1, K2, N, ctypes.c_void_p(A.data_ptr()),
                                    a_batch_stride if a_batch_stride is not None else K1 * M * K2,
                                    Wd.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    ctypes.c_void_p(C.data_ptr()), 1 if transpose_out else 0, ctypes.c_void_p(st)))
    return C


def version() -> str:
    return lib().psim_version().decode()
