"""Thin Python binding of the native MDF-LBM library (``include/mdf.h``).

Argument marshalling only: torch supplies device memory and the stream,
every step of the method runs in the library's HIP kernels.  Importing this
module loads ``libmdf.so`` and raises if it is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from .cases import CaseSpec

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmdf.so")

# enums of mdf.h
OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, ESTATE = 0, -1, -2, -3, -4, -5
D2Q5, D3Q7 = 0, 1
D2Q4, D3Q6 = 4, 5      # lattices without a rest population
D2Q9, D3Q15 = 8, 9     # lattices with diagonal links
D2Q9_Q5, D3Q15_Q7 = 12, 13   # a lattice per set (set a = 0 on D2Q5 / D3Q7)
_NQ = {D2Q5: 5, D3Q7: 7, D2Q4: 4, D3Q6: 6, D2Q9: 9, D3Q15: 15, D2Q9_Q5: 9, D3Q15_Q7: 15}
F64, F32, F16DEV, BF16DEV = 0, 1, 2, 3
PERIODIC, WALL = 0, 1
FIELD_MOMENTS, FIELD_GRAD, FIELD_DIV, FIELD_STRAIN, FIELD_STRESS, FIELD_VORT = 1, 2, 4, 8, 16, 32
FIELD_ALL = 0x3F
FIELD_ACCUMULATE = 0x40        # with step_emit / run_steady: every step adds its fields to `out`
INIT_REST, INIT_FIELDS, INIT_FIELDS_GRAD, INIT_POPULATIONS = 0, 1, 2, 3

STORAGE_NAMES = {"f64": F64, "f32": F32, "f16dev": F16DEV, "bf16dev": BF16DEV}

EXPORTED = ["mdf_workspace_size", "mdf_init", "mdf_step", "mdf_step_emit", "mdf_moments",
            "mdf_gradients", "mdf_populations", "mdf_check", "mdf_run_steady", "mdf_invariants",
            "mdf_set_launch", "mdf_set_active", "mdf_set_force_field", "mdf_autotune", "mdf_time",
            "mdf_last_error", "mdf_state_size", "mdf_save", "mdf_load",
            "mdf_graph_stats", "mdf_population_buffer", "mdf_destroy"]


class MdfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mdf status {status}: {msg}")
        self.status = status


class MdfCase(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("s0", ctypes.c_double), ("s1", ctypes.c_double), ("s2", ctypes.c_double),
        ("bc", ctypes.c_int32 * 6),
        ("wall_u", (ctypes.c_double * 3) * 6),
        ("force", ctypes.c_double * 3),
        ("R", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("u_ref", ctypes.c_double),
        ("forcing", ctypes.c_int32),
    ]


_LIB = None


def lib():
    """Load libmdf.so once; raise if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not built: run python paper_2108_08591_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, cp = ctypes.c_void_p, ctypes.POINTER(MdfCase)
        i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.mdf_workspace_size.argtypes = [i32, i32, cp, i32, i32]
        L.mdf_workspace_size.restype = ctypes.c_size_t
        L.mdf_init.argtypes = [ctypes.POINTER(vp), i32, i32, cp, i32, vp, ctypes.c_size_t,
                               ctypes.POINTER(vp), i32, ctypes.POINTER(vp), vp]
        L.mdf_step.argtypes = [vp, i32, vp]
        L.mdf_step_emit.argtypes = [vp, i32, ctypes.c_uint32, ctypes.POINTER(vp), vp]
        L.mdf_moments.argtypes = [vp, i32, vp, vp]
        L.mdf_gradients.argtypes = [vp, i32, ctypes.c_uint32, vp, vp]
        L.mdf_populations.argtypes = [vp, i32, vp, vp]
        L.mdf_check.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(i32), vp]
        L.mdf_run_steady.argtypes = [vp, dbl, i32, i64, ctypes.c_uint32, ctypes.POINTER(vp),
                                     ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(dbl), vp]
        L.mdf_invariants.argtypes = [vp, i32, ctypes.POINTER(dbl), vp]
        L.mdf_set_launch.argtypes = [vp, i32, i32, i32, i32]
        L.mdf_autotune.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl), vp]
        L.mdf_set_active.argtypes = [vp, ctypes.POINTER(i32)]
        L.mdf_set_force_field.argtypes = [vp, i32, vp]
        L.mdf_state_size.argtypes = [vp]
        L.mdf_state_size.restype = ctypes.c_size_t
        L.mdf_save.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.mdf_load.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.mdf_graph_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_char_p)]
        L.mdf_population_buffer.argtypes = [vp, i32, i32, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_size_t)]
        L.mdf_time.argtypes = [vp, i32]
        L.mdf_time.restype = i64
        L.mdf_last_error.argtypes = [vp]
        L.mdf_last_error.restype = ctypes.c_char_p
        L.mdf_destroy.argtypes = [vp]
        for name in ("mdf_init", "mdf_step", "mdf_step_emit", "mdf_moments", "mdf_gradients",
                     "mdf_populations", "mdf_check", "mdf_run_steady", "mdf_invariants",
                     "mdf_set_launch", "mdf_set_active", "mdf_set_force_field", "mdf_autotune", "mdf_destroy",
                     "mdf_save", "mdf_load", "mdf_graph_stats", "mdf_population_buffer"):
            getattr(L, name).restype = ctypes.c_int
        _LIB = L
    return _LIB


def field_layout(d: int, fields: int) -> List[tuple]:
    """(name, channels) of every selected field, in output order."""
    nsym = d * (d + 1) // 2
    out = []
    if fields & FIELD_MOMENTS:
        out.append(("ubar", d + 1))
        out.append(("P", 1))
    if fields & FIELD_GRAD:
        out.append(("grad", d * d))
    if fields & FIELD_DIV:
        out.append(("div", 1))
    if fields & FIELD_STRAIN:
        out.append(("S", nsym))
    if fields & FIELD_STRESS:
        out.append(("sigma", nsym))
    if fields & FIELD_VORT:
        out.append(("vort", 1 if d == 2 else 3))
    return out


def n_channels(d: int, fields: int) -> int:
    return sum(c for _, c in field_layout(d, fields))


def split_fields(d: int, fields: int, t: torch.Tensor) -> Dict[str, torch.Tensor]:
    """Split a channel-major output into named fields (views)."""
    res, k = {}, 0
    for name, c in field_layout(d, fields):
        v = t[k:k + c]
        if name == "grad":
            v = v.reshape((d, d) + tuple(t.shape[1:]))
        elif name in ("P", "div") or (name == "vort" and d == 2):
            v = v[0]
        res[name] = v
        k += c
    if "ubar" in res:
        res["u"] = res["ubar"][1:]
    return res


def _case_struct(spec: CaseSpec, u_ref: float = 0.0) -> MdfCase:
    c = MdfCase()
    shape = tuple(spec.shape) + ((1,) if len(spec.shape) == 2 else ())
    c.nx, c.ny, c.nz = (int(v) for v in shape)
    c.s0, c.s1, c.s2 = float(spec.s0), float(spec.s1), float(spec.s2)
    wall = spec.wall_velocity()
    for f in range(6):
        c.bc[f] = int(spec.bc[f])
        for b in range(3):
            c.wall_u[f][b] = float(wall[f, b])
    for b in range(3):
        c.force[b] = float(spec.force[b]) if b < len(spec.force) else 0.0
    c.R = float(spec.R)
    c.rho0 = float(spec.rho0)
    c.u_ref = float(u_ref)
    c.forcing = int(spec.forcing)
    return c


def _check(status, ctx=None):
    if status != OK:
        msg = lib().mdf_last_error(ctx).decode(errors="replace")
        raise MdfError(status, msg)


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Solver:
    """A context over one or more independent cases of one lattice/storage.

    ``init`` is ``"rest"`` or a tuple ``(kind, [tensor per case])`` with kind
    in {"fields", "fields_grad", "populations"}; tensors are channel-major in
    the compute dtype (FP64 for f64 storage, FP32 otherwise).  ``sets`` is
    "all" (the d + 1 sets a = 0..d) or "velocity" (only a = 1..d, the *_V
    lattices: same velocity, pressure and derived fields, fewer bytes)."""

    def __init__(self, specs: Sequence[CaseSpec], storage="f32", solid=None, init="rest",
                 u_ref: float = 0.0, device="cuda:0", stream=None, sets: str = "all"):
        if isinstance(specs, CaseSpec):
            specs = [specs]
        self.specs = list(specs)
        self.lattice = self.specs[0].lattice
        if any(s.lattice != self.lattice for s in self.specs):
            raise ValueError("all cases of a context share one lattice")
        self.storage = STORAGE_NAMES[storage] if isinstance(storage, str) else int(storage)
        self.d = self.specs[0].d
        self.q = _NQ[self.lattice]
        if sets not in ("all", "velocity"):
            raise ValueError("sets must be 'all' or 'velocity'")
        self.nsets = self.d + 1 if sets == "all" else self.d
        if sets == "velocity":
            if self.lattice in (D2Q9_Q5, D3Q15_Q7):
                raise ValueError("a lattice per set differs only in the set a = 0: use D2Q9 / D3Q15 "
                                 "with sets='velocity'")
            self.lattice += 2          # the *_V lattice ids
        self.device = torch.device(device)
        self.dtype = torch.float64 if self.storage == F64 else torch.float32
        self.stream = stream
        n = len(self.specs)
        self._cases = (MdfCase * n)(*[_case_struct(s, u_ref) for s in self.specs])
        L = lib()
        has_solid = solid is not None and any(m is not None for m in solid)
        ws = L.mdf_workspace_size(self.lattice, self.storage, self._cases, n, int(has_solid))
        if ws == 0:
            _check(EINVAL, None)
        self.workspace = torch.empty(int(ws), dtype=torch.uint8, device=self.device)
        keep = []
        solid_ptrs = None
        if has_solid:
            arr = (ctypes.c_void_p * n)()
            for k, m in enumerate(solid):
                if m is None:
                    arr[k] = None
                    continue
                t = torch.as_tensor(np.asarray(m, dtype=np.uint8) if not torch.is_tensor(m) else m)
                t = t.to(device=self.device, dtype=torch.uint8).contiguous()
                if t.numel() != self.specs[k].nodes:
                    raise ValueError(f"solid mask of case {k} has {t.numel()} entries")
                keep.append(t)
                arr[k] = t.data_ptr()
            solid_ptrs = arr
        kind, data_ptrs = INIT_REST, None
        if init != "rest":
            kname, tensors = init
            kind = {"fields": INIT_FIELDS, "fields_grad": INIT_FIELDS_GRAD,
                    "populations": INIT_POPULATIONS}[kname]
            arr = (ctypes.c_void_p * n)()
            for k, t in enumerate(tensors):
                t = torch.as_tensor(t).to(device=self.device, dtype=self.dtype).contiguous()
                need = self._init_channels(kind) * self.specs[k].nodes
                if t.numel() != need:
                    raise ValueError(f"init data of case {k}: {t.numel()} values, {need} expected")
                keep.append(t)
                arr[k] = t.data_ptr()
            data_ptrs = arr
        self._ctx = ctypes.c_void_p()
        st = L.mdf_init(ctypes.byref(self._ctx), self.lattice, self.storage, self._cases, n,
                        ctypes.c_void_p(self.workspace.data_ptr()), ctypes.c_size_t(int(ws)),
                        solid_ptrs, kind, data_ptrs, _stream_ptr(self.stream))
        _check(st, None)
        # inputs are read on the stream's timeline: keep them until it passes
        self._sync()
        del keep

    def _init_channels(self, kind):
        d = self.d
        if kind == INIT_FIELDS:
            return 1 + d
        if kind == INIT_FIELDS_GRAD:
            return 1 + d + d * d
        return self.nsets * self.q

    def _sync(self):
        (self.stream or torch.cuda.current_stream()).synchronize()

    def _handoff(self, *tensors):
        """Outputs written on the solver's own stream become safe to use on
        torch's current stream (and are kept alive for the allocator)."""
        if self.stream is None:
            return
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)
            for t in tensors:
                t.record_stream(self.stream)

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value:
            try:
                lib().mdf_destroy(ctx)
            except Exception:
                pass
            self._ctx = None

    # -------------------------------------------------------------- stepping
    def set_launch(self, bx: int, by: int, groups: int = 8, form: int = 0):
        """Tile of bx x by threads, XCD bands, and the step-kernel form: 0 one
        node per thread, 1 vector (several x-nodes per thread), 2 two steps
        per launch (2D lattices with axis links)."""
        _check(lib().mdf_set_launch(self._ctx, bx, by, groups, int(form)), self._ctx)

    def set_force_field(self, force, case: int = 0):
        """Per-node force F_b(x), array [d, *fshape] (or None to remove it);
        kept on the device by the solver for as long as it is set."""
        if force is None:
            self._force = getattr(self, "_force", {})
            self._force.pop(case, None)
            _check(lib().mdf_set_force_field(self._ctx, case, None), self._ctx)
            return
        t = torch.as_tensor(force).to(device=self.device, dtype=self.dtype).contiguous()
        if t.numel() != self.d * self.specs[case].nodes:
            raise ValueError(f"force field of case {case}: {t.numel()} values, {self.d * self.specs[case].nodes} expected")
        self._force = getattr(self, "_force", {})
        self._force[case] = t
        torch.cuda.current_stream().synchronize()
        _check(lib().mdf_set_force_field(self._ctx, case, ctypes.c_void_p(t.data_ptr())), self._ctx)

    def state_size(self) -> int:
        return int(lib().mdf_state_size(self._ctx))

    def save(self, device=None) -> torch.Tensor:
        """The solver's state (mdf_save) as a uint8 tensor on `device` (the
        solver's device by default; "cpu" gives pinned host memory)."""
        n = self.state_size()
        dev = self.device if device is None else torch.device(device)
        if dev.type == "cpu":
            blob = torch.empty(n, dtype=torch.uint8, pin_memory=True)
        else:
            blob = torch.empty(n, dtype=torch.uint8, device=dev)
        self._handoff(blob)
        _check(lib().mdf_save(self._ctx, ctypes.c_void_p(blob.data_ptr()), n, _stream_ptr(self.stream)),
               self._ctx)
        return blob

    def load(self, blob: torch.Tensor):
        """Restore a state written by save() (any device; copied to the
        solver's device first when it is in pageable host memory)."""
        b = blob.contiguous()
        if b.device.type == "cpu" and not b.is_pinned():
            b = b.to(self.device)
            torch.cuda.current_stream(self.device).synchronize()
        _check(lib().mdf_load(self._ctx, ctypes.c_void_p(b.data_ptr()), b.numel(), _stream_ptr(self.stream)),
               self._ctx)

    def set_active(self, active):
        """Enable (non-zero) or disable (0) each case."""
        arr = (ctypes.c_int32 * len(self.specs))(*[int(bool(a)) for a in active])
        _check(lib().mdf_set_active(self._ctx, arr), self._ctx)

    def autotune(self, trial_steps: int = 20):
        """Pick the fastest launch shape on real steps (advances time)."""
        chosen = (ctypes.c_int32 * 4)()
        best = ctypes.c_double()
        _check(lib().mdf_autotune(self._ctx, int(trial_steps), chosen, ctypes.byref(best),
                                  _stream_ptr(self.stream)), self._ctx)
        return tuple(chosen[:]), best.value

    def step(self, nsteps: int = 1):
        _check(lib().mdf_step(self._ctx, int(nsteps), _stream_ptr(self.stream)), self._ctx)

    def new_field_buffers(self, fields: int) -> List[torch.Tensor]:
        nch = n_channels(self.d, fields)
        return [torch.empty((nch,) + s.fshape, dtype=self.dtype, device=self.device)
                for s in self.specs]

    def step_emit(self, nsteps: int, fields: int, out: Optional[List[torch.Tensor]] = None):
        if out is None:
            out = self.new_field_buffers(fields)
        arr = (ctypes.c_void_p * len(out))(*[t.data_ptr() for t in out])
        _check(lib().mdf_step_emit(self._ctx, int(nsteps), int(fields), arr,
                                   _stream_ptr(self.stream)), self._ctx)
        self._handoff(*out)
        return out

    def time(self, case: int = 0) -> int:
        return int(lib().mdf_time(self._ctx, case))

    def graph_stats(self) -> Dict[str, object]:
        """Chunks captured as HIP graphs, replayed, run as plain launches,
        failed captures and the last capture error (mdf_graph_stats)."""
        stats = (ctypes.c_int64 * 4)()
        msg = ctypes.c_char_p()
        _check(lib().mdf_graph_stats(self._ctx, stats, ctypes.byref(msg)), self._ctx)
        return {"captured": stats[0], "replayed": stats[1], "plain": stats[2], "failed": stats[3],
                "error": (msg.value or b"").decode(errors="replace")}

    def population_buffer(self, which: int, case: int = 0) -> torch.Tensor:
        """The raw bytes of population buffer `which` of a case
        (mdf_population_buffer) as a uint8 view of the workspace: 0 holds
        f*(t), 1 is the buffer the next step overwrites."""
        ptr = ctypes.c_void_p()
        nbytes = ctypes.c_size_t()
        _check(lib().mdf_population_buffer(self._ctx, case, int(which), ctypes.byref(ptr), ctypes.byref(nbytes)),
               self._ctx)
        off = int(ptr.value) - self.workspace.data_ptr()
        return self.workspace[off: off + int(nbytes.value)]

    # -------------------------------------------------------------- read-outs
    def gradients(self, fields: int, case: int = 0) -> torch.Tensor:
        out = torch.empty((n_channels(self.d, fields),) + self.specs[case].fshape, dtype=self.dtype,
                          device=self.device)
        _check(lib().mdf_gradients(self._ctx, case, int(fields), ctypes.c_void_p(out.data_ptr()),
                                   _stream_ptr(self.stream)), self._ctx)
        self._handoff(out)
        return out

    def moments(self, case: int = 0) -> torch.Tensor:
        out = torch.empty((self.d + 2,) + self.specs[case].fshape, dtype=self.dtype, device=self.device)
        _check(lib().mdf_moments(self._ctx, case, ctypes.c_void_p(out.data_ptr()),
                                 _stream_ptr(self.stream)), self._ctx)
        self._handoff(out)
        return out

    def fields(self, fields: int = FIELD_ALL, case: int = 0) -> Dict[str, torch.Tensor]:
        return split_fields(self.d, fields, self.gradients(fields, case))

    def populations(self, case: int = 0) -> torch.Tensor:
        out = torch.empty((self.nsets, self.q) + self.specs[case].fshape, dtype=self.dtype,
                          device=self.device)
        _check(lib().mdf_populations(self._ctx, case, ctypes.c_void_p(out.data_ptr()),
                                     _stream_ptr(self.stream)), self._ctx)
        self._handoff(out)
        return out

    def check(self):
        n = len(self.specs)
        res = (ctypes.c_double * n)()
        status = (ctypes.c_int32 * n)()
        st = lib().mdf_check(self._ctx, res, status, _stream_ptr(self.stream))
        if st not in (OK, EUNSTABLE):
            _check(st, self._ctx)
        return np.array(res[:]), np.array(status[:])

    def run_steady(self, tol: float = 1e-8, K: int = 100, max_steps: int = 10 ** 7, fields: int = 0,
                   out: Optional[List[torch.Tensor]] = None):
        n = len(self.specs)
        status = (ctypes.c_int32 * n)()
        steps = (ctypes.c_int64 * n)()
        res = (ctypes.c_double * n)()
        arr = None
        if fields:
            if out is None:
                raise ValueError("fields selected without output buffers")
            arr = (ctypes.c_void_p * n)(*[t.data_ptr() for t in out])
        st = lib().mdf_run_steady(self._ctx, float(tol), int(K), int(max_steps), int(fields), arr,
                                  status, steps, res, _stream_ptr(self.stream))
        if st not in (OK, EUNSTABLE):
            _check(st, self._ctx)
        return np.array(status[:]), np.array(steps[:]), np.array(res[:])

    def invariants(self, case: int = 0) -> np.ndarray:
        out = (ctypes.c_double * (self.d + 2))()
        st = lib().mdf_invariants(self._ctx, case, out, _stream_ptr(self.stream))
        if st not in (OK, EUNSTABLE):
            _check(st, self._ctx)
        return np.array(out[:])
