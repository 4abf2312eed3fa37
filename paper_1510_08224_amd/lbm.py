"""Thin ctypes binding of ``include/lbm.h`` (argument marshalling only).

Every function named ``lbm_*`` here calls the C entry point of the same name
in ``liblbm.so`` and raises :class:`LbmError` on a negative return code.
:class:`Solver` bundles a handle with those calls.  Device memory for the
population buffers can come from PyTorch (``torch_memory=True``), and the
solver can run on a PyTorch stream; nothing else of PyTorch is used.  All
arithmetic of the method runs in the library's HIP kernels; there is no
fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lbm.h")

LBM_OK, LBM_ERR_ARG, LBM_ERR_NOMEM, LBM_ERR_DEVICE = 0, -1, -2, -3
LBM_ERR_STATE, LBM_ERR_UNSTABLE, LBM_ERR_UNSUPPORTED = -4, -5, -6
LBM_F64, LBM_F32, LBM_F16 = 0, 1, 2
LBM_LEFT, LBM_RIGHT, LBM_BOTTOM, LBM_TOP = 0, 1, 2, 3
LBM_BC_PERIODIC, LBM_BC_WALL, LBM_BC_NEE = 0, 1, 2
LBM_T_PERIODIC, LBM_T_DIRICHLET, LBM_T_ADIABATIC, LBM_T_NEE_DIRICHLET, LBM_T_NEE_ADIABATIC = 0, 1, 2, 3, 4

LBM_MODEL_D2Q5, LBM_MODEL_D2Q9T, LBM_MODEL_ISOTHERMAL = 0, 1, 2
LBM_POLICY_DEFAULT, LBM_POLICY_KEEP, LBM_POLICY_XCD_BANDS, LBM_POLICY_KEEP_STORES = -2, -1, 1, 2
LBM_POLICY_XCD_STRIPS, LBM_POLICY_FUSE2, LBM_POLICY_FUSEK = 4, 8, 16
LBM_COLLISION_MRT, LBM_COLLISION_BGK, LBM_COLLISION_ORTHO_MRT = 0, 1, 2
STORAGE = {"f64": LBM_F64, "f32": LBM_F32, "f16": LBM_F16}
MODEL = {"d2q5": LBM_MODEL_D2Q5, "d2q9t": LBM_MODEL_D2Q9T, "isothermal": LBM_MODEL_ISOTHERMAL}
MODEL_NG = {LBM_MODEL_D2Q5: 5, LBM_MODEL_D2Q9T: 9, LBM_MODEL_ISOTHERMAL: 0}
_CODES = {-1: "LBM_ERR_ARG", -2: "LBM_ERR_NOMEM", -3: "LBM_ERR_DEVICE", -4: "LBM_ERR_STATE",
          -5: "LBM_ERR_UNSTABLE", -6: "LBM_ERR_UNSUPPORTED"}


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class LbmParams(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("reserved0", ctypes.c_uint32),
        ("ra", ctypes.c_double), ("pr", ctypes.c_double), ("u_c", ctypes.c_double),
        ("length", ctypes.c_double), ("t_hot", ctypes.c_double), ("t_cold", ctypes.c_double),
        ("s_e", ctypes.c_double), ("s_q", ctypes.c_double), ("s_eps", ctypes.c_double),
        ("zeta_e", ctypes.c_double), ("zeta_nu", ctypes.c_double), ("varpi", ctypes.c_double),
        ("zeta_q", ctypes.c_double), ("zeta_eps", ctypes.c_double), ("theta", ctypes.c_double),
        ("s_nu", ctypes.c_double), ("zeta_alpha", ctypes.c_double),
        ("ax", ctypes.c_double), ("ay", ctypes.c_double),
        ("bc_flow", ctypes.c_int32 * 4), ("bc_temp", ctypes.c_int32 * 4),
        ("collision", ctypes.c_int32), ("reserved1", ctypes.c_int32),
        ("wall_T", ctypes.c_double * 4), ("wall_u", (ctypes.c_double * 2) * 4),
    ]


_lib = None
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_SIGS = {
    "lbm_params_default": (None, [ctypes.POINTER(LbmParams)]),
    "lbm_abi_version": (ctypes.c_int32, []),
    "lbm_rate_for_reynolds": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double, _D]),
    "lbm_build_info": (ctypes.c_char_p, []),
    "lbm_required_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "lbm_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, _P]),
    "lbm_create_ext": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, _P, ctypes.c_uint64, _P]),
    "lbm_set_params": (ctypes.c_int, [_P, ctypes.POINTER(LbmParams)]),
    "lbm_get_derived": (ctypes.c_int, [_P, _D, _D, _D, _D, _D, _D]),
    "lbm_init_temperature": (ctypes.c_int, [_P, _D]),
    "lbm_step": (ctypes.c_int, [_P, ctypes.c_int64]),
    "lbm_time": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "lbm_synchronize": (ctypes.c_int, [_P]),
    "lbm_moments": (ctypes.c_int, [_P, _D, _D, _D, _D]),
    "lbm_moments_device": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "lbm_nusselt": (ctypes.c_int, [_P, ctypes.c_int32, _D, _D, ctypes.POINTER(ctypes.c_int32)]),
    "lbm_nusselt_local": (ctypes.c_int, [_P, ctypes.c_int32, _D]),
    "lbm_residual": (ctypes.c_int, [_P, _D, ctypes.POINTER(ctypes.c_int64)]),
    "lbm_residual_static": (ctypes.c_int, [_P, _D, ctypes.POINTER(ctypes.c_int64)]),
    "lbm_get_populations": (ctypes.c_int, [_P, _D, _D]),
    "lbm_set_populations": (ctypes.c_int, [_P, _D, _D]),
    "lbm_state_bytes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint64)]),
    "lbm_save_state": (ctypes.c_int, [_P, _P, ctypes.c_uint64]),
    "lbm_load_state": (ctypes.c_int, [_P, _P, ctypes.c_uint64]),
    "lbm_stream": (_P, [_P]),
    "lbm_storage_of": (ctypes.c_int32, [_P]),
    "lbm_model_of": (ctypes.c_int32, [_P]),
    "lbm_set_launch": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "lbm_get_launch": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "lbm_set_graph_steps": (ctypes.c_int, [_P, ctypes.c_int32]),
    "lbm_get_graph_steps": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "lbm_steps_per_launch": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "lbm_batch_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int32, _P]),
    "lbm_batch_add": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_int32)]),
    "lbm_batch_remove": (ctypes.c_int, [_P, ctypes.c_int32]),
    "lbm_batch_size": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "lbm_batch_member": (_P, [_P, ctypes.c_int32]),
    "lbm_batch_step": (ctypes.c_int, [_P, ctypes.c_int64]),
    "lbm_batch_set_graph_steps": (ctypes.c_int, [_P, ctypes.c_int32]),
    "lbm_batch_set_policy": (ctypes.c_int, [_P, ctypes.c_int32]),
    "lbm_batch_set_tuning": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "lbm_batch_get_tuning": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32)]),
    "lbm_batch_steps_per_launch": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "lbm_batch_synchronize": (ctypes.c_int, [_P]),
    "lbm_batch_residual": (ctypes.c_int, [_P, _D, ctypes.POINTER(ctypes.c_int64)]),
    "lbm_batch_stream": (_P, [_P]),
    "lbm_batch_last_error": (ctypes.c_char_p, [_P]),
    "lbm_batch_destroy": (None, [_P]),
    "lbm_last_error": (ctypes.c_char_p, [_P]),
    "lbm_destroy": (None, [_P]),
}


def lib():
    """The loaded HIP library.  Raises if it has not been built: there is no
    other implementation to fall back to."""
    global _lib
    if _lib is None:
        # PyTorch's wheel ships its own libamdhip64 under the same soname as
        # /opt/rocm's.  Loading torch first makes liblbm.so bind to that one
        # runtime, so torch tensors and streams and the library share it;
        # loading liblbm.so first would bring up a second HIP runtime in the
        # process, after which torch cannot open the GPU.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1510_08224_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_symbols() -> list[str]:
    """Names of the functions declared in include/lbm.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_\w+)\s*\(", txt)))


def _check(rc: int, h=None):
    if rc != LBM_OK:
        msg = lib().lbm_last_error(h)
        raise LbmError(rc, msg.decode() if msg else "")
    return rc


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def lbm_params_default() -> LbmParams:
    p = LbmParams()
    lib().lbm_params_default(ctypes.byref(p))
    return p


def lbm_rate_for_reynolds(re: float, length: float, u: float) -> float:
    """s_nu for a Reynolds number (the library's rate map of Sec. 3.2)."""
    s = ctypes.c_double()
    _check(lib().lbm_rate_for_reynolds(float(re), float(length), float(u), ctypes.byref(s)))
    return s.value


def lbm_params_from_problem(pb) -> LbmParams:
    """Marshal a ``workloads.Problem`` into ``lbm_params``."""
    p = lbm_params_default()
    for k in ("ra", "pr", "u_c", "length", "t_hot", "t_cold", "s_e", "s_q", "s_eps", "zeta_e",
              "zeta_nu", "varpi", "s_nu", "zeta_alpha", "ax", "ay", "zeta_q", "zeta_eps", "theta"):
        setattr(p, k, float(getattr(pb, k)))
    for s in range(4):
        p.bc_flow[s] = int(pb.bc_flow[s])
        p.bc_temp[s] = int(pb.bc_temp[s])
        p.wall_T[s] = float(pb.wall_T[s])
        p.wall_u[s][0] = float(pb.wall_u[s][0])
        p.wall_u[s][1] = float(pb.wall_u[s][1])
    p.collision = int(getattr(pb, "collision", LBM_COLLISION_MRT))
    return p


def lbm_required_bytes(nx: int, ny: int, storage: int, model: int = LBM_MODEL_D2Q5) -> int:
    b = ctypes.c_uint64()
    _check(lib().lbm_required_bytes(nx, ny, storage, model, ctypes.byref(b)))
    return b.value


def lbm_create(nx: int, ny: int, storage: int, model: int = LBM_MODEL_D2Q5, stream=None):
    h = _P()
    _check(lib().lbm_create(ctypes.byref(h), nx, ny, storage, model, stream))
    return h


def lbm_create_ext(nx: int, ny: int, storage: int, model: int, device_ptr: int, nbytes: int, stream=None):
    h = _P()
    _check(lib().lbm_create_ext(ctypes.byref(h), nx, ny, storage, model, _P(device_ptr), nbytes, stream))
    return h


def lbm_destroy(h):
    lib().lbm_destroy(h)


class Solver:
    """One lattice on the current GPU.  ``storage`` is "f64", "f32" or
    "f16".  With ``torch_memory`` the population buffers are a PyTorch
    allocation (kept alive by the solver) and the solver launches on the
    current PyTorch stream."""

    def __init__(self, nx: int, ny: int, storage: str = "f64", torch_memory: bool = False, stream=None,
                 model="d2q5"):
        self.nx, self.ny = int(nx), int(ny)
        self.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        self.model = MODEL[model] if isinstance(model, str) else int(model)
        self.ng = MODEL_NG[self.model]
        self._mem = None
        self.h = None
        self._owner = None     # the Batch whose stream this solver launches on
        if torch_memory:
            import torch
            nbytes = lbm_required_bytes(self.nx, self.ny, self.storage, self.model)
            self._mem = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            ptr = self._mem.data_ptr()
            ptr = (ptr + 255) // 256 * 256
            if stream is None:
                stream = torch.cuda.current_stream().cuda_stream or None
            self.h = lbm_create_ext(self.nx, self.ny, self.storage, self.model, ptr, nbytes, stream)
        else:
            self.h = lbm_create(self.nx, self.ny, self.storage, self.model, stream)

    @property
    def model_name(self) -> str:
        return {v: k for k, v in MODEL.items()}[self.model]

    def close(self):
        if self.h:
            lbm_destroy(self.h)
            self.h = None
        self._mem = None
        if self._owner is not None:
            owner, self._owner = self._owner, None
            owner._solver_closed(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- problem ---------------------------------------------------------
    def set_params(self, pb_or_params):
        p = pb_or_params if isinstance(pb_or_params, LbmParams) else lbm_params_from_problem(pb_or_params)
        _check(lib().lbm_set_params(self.h, ctypes.byref(p)), self.h)

    def derived(self) -> dict:
        s9 = np.zeros(9); q9 = np.zeros(9)
        gb, t0, ln, dt = (ctypes.c_double() for _ in range(4))
        _check(lib().lbm_get_derived(self.h, _dp(s9), _dp(q9), ctypes.byref(gb), ctypes.byref(t0),
                                     ctypes.byref(ln), ctypes.byref(dt)), self.h)
        return {"s": s9, "q": q9[:self.ng], "gbeta": gb.value, "T0": t0.value, "length": ln.value,
                "dT": dt.value}

    def init_temperature(self, T=None):
        if T is not None:
            T = np.ascontiguousarray(T, dtype=np.float64).reshape(self.ny, self.nx)
        _check(lib().lbm_init_temperature(self.h, _dp(T)), self.h)

    def set_launch(self, block_x=0, block_y=0, rows=0, policy=LBM_POLICY_KEEP):
        _check(lib().lbm_set_launch(self.h, block_x, block_y, rows, policy), self.h)

    def get_launch(self):
        """(block_x, block_y, rows_per_thread, policy mask)."""
        a, b, c, d = (ctypes.c_int32() for _ in range(4))
        _check(lib().lbm_get_launch(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)),
               self.h)
        return a.value, b.value, c.value, d.value

    @property
    def steps_per_launch(self) -> int:
        """Time steps per step-kernel launch (2 with fused pairs)."""
        v = ctypes.c_int32()
        _check(lib().lbm_steps_per_launch(self.h, ctypes.byref(v)), self.h)
        return v.value

    def set_graph_steps(self, steps: int):
        _check(lib().lbm_set_graph_steps(self.h, int(steps)), self.h)

    def get_graph_steps(self) -> int:
        v = ctypes.c_int32()
        _check(lib().lbm_get_graph_steps(self.h, ctypes.byref(v)), self.h)
        return v.value

    # -- time stepping ---------------------------------------------------
    def step(self, n: int = 1):
        _check(lib().lbm_step(self.h, int(n)), self.h)

    @property
    def time(self) -> int:
        t = ctypes.c_int64()
        _check(lib().lbm_time(self.h, ctypes.byref(t)), self.h)
        return t.value

    def synchronize(self):
        _check(lib().lbm_synchronize(self.h), self.h)

    @property
    def stream(self):
        return lib().lbm_stream(self.h)

    # -- readouts --------------------------------------------------------
    def moments(self):
        shp = (self.ny, self.nx)
        out = [np.zeros(shp) for _ in range(4)]
        _check(lib().lbm_moments(self.h, *(_dp(a) for a in out)), self.h)
        return tuple(out)

    def moments_device(self, rho=None, ux=None, uy=None, T=None):
        """Fill caller-owned device arrays (e.g. float64 torch tensors of nx*ny)."""
        ptr = lambda t: None if t is None else _P(t.data_ptr())
        _check(lib().lbm_moments_device(self.h, ptr(rho), ptr(ux), ptr(uy), ptr(T)), self.h)

    def nusselt(self, side: int):
        m, x = ctypes.c_double(), ctypes.c_double()
        i = ctypes.c_int32()
        _check(lib().lbm_nusselt(self.h, side, ctypes.byref(m), ctypes.byref(x), ctypes.byref(i)), self.h)
        return m.value, x.value, i.value

    def nusselt_local(self, side: int):
        n = self.ny if side in (LBM_LEFT, LBM_RIGHT) else self.nx
        out = np.zeros(n)
        _check(lib().lbm_nusselt_local(self.h, side, _dp(out)), self.h)
        return out

    def residual(self, raise_unstable: bool = True):
        r = ctypes.c_double()
        bad = ctypes.c_int64()
        rc = lib().lbm_residual(self.h, ctypes.byref(r), ctypes.byref(bad))
        if rc != LBM_OK and (rc != LBM_ERR_UNSTABLE or raise_unstable):
            _check(rc, self.h)
        return r.value, bad.value

    def residual_static(self, raise_unstable: bool = True):
        """lbm_residual_static: the residual without allocating device memory
        (the snapshot must exist: one residual() call allocates it)."""
        r = ctypes.c_double()
        bad = ctypes.c_int64()
        rc = lib().lbm_residual_static(self.h, ctypes.byref(r), ctypes.byref(bad))
        if rc != LBM_OK and (rc != LBM_ERR_UNSTABLE or raise_unstable):
            _check(rc, self.h)
        return r.value, bad.value

    def get_populations(self):
        f = np.zeros((9, self.ny, self.nx)); g = np.zeros((self.ng, self.ny, self.nx))
        _check(lib().lbm_get_populations(self.h, _dp(f), _dp(g)), self.h)
        return f, g

    def set_populations(self, f, g):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(9, self.ny, self.nx)
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(self.ng, self.ny, self.nx) if self.ng else None
        _check(lib().lbm_set_populations(self.h, _dp(f), _dp(g)), self.h)

    def save_state(self) -> bytes:
        n = ctypes.c_uint64()
        _check(lib().lbm_state_bytes(self.h, ctypes.byref(n)), self.h)
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().lbm_save_state(self.h, ctypes.cast(buf, _P), n.value), self.h)
        return buf.raw

    def load_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().lbm_load_state(self.h, ctypes.cast(buf, _P), len(blob)), self.h)


def _bcheck(rc: int, b=None):
    if rc != LBM_OK:
        msg = lib().lbm_batch_last_error(b)
        raise LbmError(rc, msg.decode() if msg else "")
    return rc


class Batch:
    """A set of solvers advanced together (one launch per step for all).
    Solvers for a batch are created with :meth:`new_solver` so that they
    share its storage and stream.  The batch's stream must outlive them:
    :meth:`close` releases the batch at once when they are all closed, and
    otherwise when the last of them closes."""

    def __init__(self, storage: str = "f32", stream=None):
        self.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        self.storage_name = {v: k for k, v in STORAGE.items()}[self.storage]
        h = _P()
        _bcheck(lib().lbm_batch_create(ctypes.byref(h), self.storage, stream))
        self.h = h
        self.members: dict[int, Solver] = {}
        self._spawned: set[int] = set()   # ids of open solvers on this batch's stream
        self._closing = False

    @property
    def stream(self):
        return lib().lbm_batch_stream(self.h)

    def new_solver(self, nx: int, ny: int, torch_memory: bool = False, model="d2q5") -> Solver:
        if self._closing:
            raise RuntimeError("the batch is closed")
        S = Solver(nx, ny, self.storage, torch_memory=torch_memory, stream=self.stream, model=model)
        S._owner = self
        self._spawned.add(id(S))
        return S

    def _solver_closed(self, S: Solver):
        self._spawned.discard(id(S))
        if self._closing and not self._spawned:
            self._destroy()

    def add(self, solver: Solver) -> int:
        slot = ctypes.c_int32()
        _bcheck(lib().lbm_batch_add(self.h, solver.h, ctypes.byref(slot)), self.h)
        self.members[slot.value] = solver
        return slot.value

    def remove(self, slot: int) -> Solver:
        _bcheck(lib().lbm_batch_remove(self.h, int(slot)), self.h)
        return self.members.pop(slot)

    def size(self):
        a, s = ctypes.c_int32(), ctypes.c_int32()
        _bcheck(lib().lbm_batch_size(self.h, ctypes.byref(a), ctypes.byref(s)), self.h)
        return a.value, s.value

    def step(self, n: int = 1):
        _bcheck(lib().lbm_batch_step(self.h, int(n)), self.h)

    def set_tuning(self, xcd_order: int = -1, keep_stores: int = -1, largest_first: int = 0):
        _bcheck(lib().lbm_batch_set_tuning(self.h, int(xcd_order), int(keep_stores), int(largest_first)), self.h)

    def get_tuning(self) -> dict:
        o, k, l = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _bcheck(lib().lbm_batch_get_tuning(self.h, ctypes.byref(o), ctypes.byref(k), ctypes.byref(l)), self.h)
        return {"xcd_order": o.value, "keep_stores": k.value, "largest_first": l.value}

    def set_graph_steps(self, steps: int):
        _bcheck(lib().lbm_batch_set_graph_steps(self.h, int(steps)), self.h)

    def set_policy(self, policy: int):
        """LBM_POLICY_DEFAULT, or a mask of LBM_POLICY_FUSE2 and
        LBM_POLICY_FUSEK (0: one launch per step)."""
        _bcheck(lib().lbm_batch_set_policy(self.h, int(policy)), self.h)

    @property
    def steps_per_launch(self) -> int:
        v = ctypes.c_int32()
        _bcheck(lib().lbm_batch_steps_per_launch(self.h, ctypes.byref(v)), self.h)
        return v.value

    def synchronize(self):
        _bcheck(lib().lbm_batch_synchronize(self.h), self.h)

    def residual(self):
        """Per-slot residuals and non-finite counts (NaN / -1 for free slots)."""
        _, slots = self.size()
        r = np.zeros(max(slots, 1)); bad = np.zeros(max(slots, 1), dtype=np.int64)
        rc = lib().lbm_batch_residual(self.h, _dp(r), bad.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        if rc not in (LBM_OK, LBM_ERR_UNSTABLE):
            _bcheck(rc, self.h)
        return r[:slots], bad[:slots]

    def close(self):
        """Release the batch; its stream stays until every solver made by
        :meth:`new_solver` is closed."""
        self._closing = True
        if not self._spawned:
            self._destroy()

    def _destroy(self):
        if self.h:
            lib().lbm_batch_destroy(self.h)
            self.h = None
        self.members = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
