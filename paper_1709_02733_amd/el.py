"""Python binding of the elastic operator library (ctypes over libel.so).

Argument marshalling only: every step of H and H^T runs in the HIP kernels
behind include/el.h.  PyTorch supplies device memory (the caller-owned
workspace, inputs and outputs) and the stream.  If libel.so is missing the
import of this module's functions raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libel.so")

EL_OK, EL_EINVAL, EL_EUNSTABLE, EL_ERANGE, EL_ENOMEM, EL_EDEVICE, EL_EBUSY = 0, -1, -2, -3, -4, -5, -6
OP_FORWARD, OP_ADJOINT = 0, 1
EL_F32, EL_F64 = 0, 1
FIELDS = ("u1", "u2", "u3", "s11", "s22", "s33", "s23", "s13", "s12")


class ElError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{status_name(status)}: {msg}")
        self.status = status


MAX_MECH = 4


class Relaxation(ctypes.Structure):
    """el_relaxation (include/el.h): frequency-dependent absorption mechanisms."""
    _fields_ = [("nmech", ctypes.c_int32), ("omega", ctypes.c_double * MAX_MECH),
                ("weight", ctypes.c_double * MAX_MECH)]


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dt", ctypes.c_double),
                ("nsteps", ctypes.c_int32), ("npml", ctypes.c_int32),
                ("pml_R", ctypes.c_double), ("pml_npower", ctypes.c_double), ("pml_f0", ctypes.c_double),
                ("precision", ctypes.c_int32), ("relax", Relaxation)]


class FluidStats(ctypes.Structure):
    """el_fluid_stats (include/el.h)."""
    _fields_ = [("tiles", ctypes.c_int64), ("cells", ctypes.c_int64), ("layer_cells", ctypes.c_int64),
                ("skipped_stores", ctypes.c_int64), ("uniform_cells", ctypes.c_int64),
                ("column_cells", ctypes.c_int64)]


_lib = None
EXPORTS = ("el_version", "el_status_string", "el_last_error", "el_grid_check", "el_plan_bytes",
           "el_plan_create", "el_plan_destroy", "el_forward", "el_forward_energy", "el_adjoint", "el_dot_f64",
           "el_dot_f64_noalloc", "el_eir_apply",
           "el_plan_field", "el_plan_layout", "el_plan_sizes", "el_plan_relaxation", "el_plan_fluid_path",
           "el_plan_timing",
           "el_plan_kernel_time",
           "el_exec_create", "el_exec_destroy", "el_exec_start", "el_exec_poll", "el_exec_wait", "el_exec_slots",
           "el_exec_set_ahead", "el_exec_pump",
           "el_group_create", "el_group_destroy", "el_group_add", "el_group_run", "el_group_sync", "el_group_poll",
           "el_group_remove", "el_group_members")
KERNELS = ("velocity", "stress", "adj_velocity", "adj_stress", "gather", "scatter", "relax")


def lib():
    """Load libel.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1709_02733_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32
        L.el_version.restype = ctypes.c_char_p
        L.el_status_string.restype = ctypes.c_char_p
        L.el_status_string.argtypes = [st]
        L.el_last_error.restype = ctypes.c_char_p
        L.el_grid_check.restype = st
        L.el_grid_check.argtypes = [ctypes.POINTER(Grid), vp, i32]
        L.el_plan_bytes.restype = st
        L.el_plan_bytes.argtypes = [ctypes.POINTER(Grid), i32, ctypes.POINTER(ctypes.c_size_t)]
        L.el_plan_create.restype = st
        L.el_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Grid), vp, vp, vp, vp, vp, vp, i32,
                                     vp, ctypes.c_size_t, vp]
        L.el_plan_destroy.restype = st
        L.el_plan_destroy.argtypes = [vp]
        L.el_forward.restype = st
        L.el_forward.argtypes = [vp, vp, vp, vp]
        L.el_forward_energy.restype = st
        L.el_forward_energy.argtypes = [vp, vp, vp, i32, vp, vp]
        L.el_adjoint.restype = st
        L.el_adjoint.argtypes = [vp, vp, vp, vp]
        L.el_dot_f64.restype = st
        L.el_dot_f64.argtypes = [vp, i32, vp, vp, vp, vp]
        L.el_dot_f64_noalloc.restype = st
        L.el_dot_f64_noalloc.argtypes = [i32, ctypes.c_int64, vp, vp, vp, vp]
        L.el_eir_apply.restype = st
        L.el_eir_apply.argtypes = [vp, i32, vp, vp, i32, i32, i32, vp]
        L.el_plan_field.restype = st
        L.el_plan_field.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_size_t)]
        L.el_plan_layout.restype = st
        L.el_plan_layout.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int64)]
        L.el_plan_sizes.restype = st
        L.el_plan_sizes.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.el_plan_relaxation.restype = st
        L.el_plan_relaxation.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int64)]
        L.el_plan_fluid_path.restype = st
        L.el_plan_fluid_path.argtypes = [vp, i32, ctypes.POINTER(FluidStats)]
        L.el_plan_timing.restype = st
        L.el_plan_timing.argtypes = [vp, i32]
        L.el_plan_kernel_time.restype = st
        L.el_plan_kernel_time.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
        L.el_exec_create.restype = st
        L.el_exec_create.argtypes = [ctypes.POINTER(vp), i32, i32]
        L.el_exec_destroy.restype = st
        L.el_exec_destroy.argtypes = [vp]
        L.el_exec_start.restype = st
        L.el_exec_start.argtypes = [vp, vp, i32, vp, vp, vp, ctypes.POINTER(i32)]
        L.el_exec_poll.restype = st
        L.el_exec_poll.argtypes = [vp, i32, ctypes.POINTER(i32)]
        L.el_exec_wait.restype = st
        L.el_exec_wait.argtypes = [vp, i32]
        L.el_exec_slots.restype = st
        L.el_exec_slots.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.el_exec_set_ahead.restype = st
        L.el_exec_set_ahead.argtypes = [vp, i32]
        L.el_exec_pump.restype = st
        L.el_exec_pump.argtypes = [vp]
        L.el_group_create.restype = st
        L.el_group_create.argtypes = [ctypes.POINTER(vp), i32, i32]
        L.el_group_destroy.restype = st
        L.el_group_destroy.argtypes = [vp]
        L.el_group_add.restype = st
        L.el_group_add.argtypes = [vp, vp, i32, vp, vp, vp, ctypes.POINTER(i32)]
        L.el_group_run.restype = st
        L.el_group_run.argtypes = [vp, i32]
        L.el_group_sync.restype = st
        L.el_group_sync.argtypes = [vp, i32]
        L.el_group_poll.restype = st
        L.el_group_poll.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.el_group_remove.restype = st
        L.el_group_remove.argtypes = [vp, i32]
        L.el_group_members.restype = st
        L.el_group_members.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
        _lib = L
    return _lib


def status_name(s: int) -> str:
    try:
        return lib().el_status_string(s).decode()
    except RuntimeError:
        return str(s)


def _check(status: int):
    if status != EL_OK:
        raise ElError(status, lib().el_last_error().decode())


def version() -> str:
    return lib().el_version().decode()


def make_grid(nx, ny, nz, dx, dt, nsteps, npml, precision="f32", pml_R=0.0, pml_npower=0.0, pml_f0=0.0,
              mechanisms=None) -> Grid:
    """mechanisms: relaxation mechanisms of the frequency-dependent absorption as a list of
    (omega_l in rad/s, weight w_l) pairs (el_relaxation), None for the diffusive model."""
    prec = {"f32": EL_F32, "f64": EL_F64}[precision] if isinstance(precision, str) else int(precision)
    rx = Relaxation()
    mech = list(mechanisms or [])
    rx.nmech = len(mech)
    for l, (om, w) in enumerate(mech[:MAX_MECH]):
        rx.omega[l], rx.weight[l] = float(om), float(w)
    return Grid(int(nx), int(ny), int(nz), float(dx), float(dt), int(nsteps), int(npml),
                float(pml_R), float(pml_npower), float(pml_f0), prec, rx)


def grid_check(grid: Grid, rec=None) -> None:
    r = None if rec is None else np.ascontiguousarray(rec, dtype=np.float64).reshape(-1, 3)
    n = 0 if r is None else r.shape[0]
    _check(lib().el_grid_check(ctypes.byref(grid), None if r is None else r.ctypes.data_as(ctypes.c_void_p), n))


def plan_bytes(grid: Grid, nrec: int) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().el_plan_bytes(ctypes.byref(grid), int(nrec), ctypes.byref(out)))
    return int(out.value)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_f32(a, device):
    t = torch.as_tensor(a)
    return t.to(device=device, dtype=torch.float32).contiguous()


class Plan:
    """One grid, medium and receiver set on one GPU; applies H and H^T.

    lam, mu, rho, alpha: cell maps [nz][ny][nx] (numpy or torch); they are
    copied into the plan's workspace.  rec: [L][3] receiver positions in
    metres from the centre of cell (0,0,0).
    """

    def __init__(self, nx, ny, nz, dx, dt, nsteps, npml, lam, mu, rho, alpha, rec,
                 precision="f32", pml_R=0.0, pml_npower=0.0, pml_f0=0.0, device=None, stream=None,
                 alpha_r=None, mechanisms=None):
        """alpha_r, mechanisms: frequency-dependent absorption (el_relaxation): the strength
        cell map (1/s) and the (omega_l, w_l) pairs of the relaxation mechanisms."""
        L = lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.grid = make_grid(nx, ny, nz, dx, dt, nsteps, npml, precision, pml_R, pml_npower, pml_f0,
                              mechanisms=mechanisms)
        self.nmech = int(self.grid.relax.nmech)
        self.precision = "f64" if self.grid.precision == EL_F64 else "f32"
        self.dtype = torch.float64 if self.precision == "f64" else torch.float32
        self.shape = (int(nz), int(ny), int(nx))
        self.N = int(nx) * int(ny) * int(nz)
        self.nsteps = int(nsteps)
        rec = np.ascontiguousarray(np.asarray(rec, dtype=np.float64).reshape(-1, 3))
        self.nrec = rec.shape[0]
        self._rec = rec
        self.bytes = plan_bytes(self.grid, self.nrec)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(self.bytes, dtype=torch.uint8, device=self.device)
            maps = [_dev_f32(m, self.device) for m in (lam, mu, rho, alpha)]
            ar = _dev_f32(alpha_r, self.device) if self.nmech > 0 and alpha_r is not None else None
            for m in maps + ([ar] if ar is not None else []):
                assert m.numel() == self.N, "material map size does not match the grid"
            h = ctypes.c_void_p(None)
            st = L.el_plan_create(ctypes.byref(h), ctypes.byref(self.grid),
                                  *[ctypes.c_void_p(m.data_ptr()) for m in maps],
                                  ctypes.c_void_p(ar.data_ptr() if ar is not None else None),
                                  rec.ctypes.data_as(ctypes.c_void_p), self.nrec,
                                  ctypes.c_void_p(self.workspace.data_ptr()), self.bytes, _stream(stream))
            _check(st)
        self._h = h
        self._lib = lib()

    @classmethod
    def from_scenario(cls, sc, precision="f32", **kw):
        if getattr(sc, "mechanisms", None) and "mechanisms" not in kw:
            kw.update(alpha_r=sc.alpha_r, mechanisms=sc.mechanisms)
        return cls(sc.nx, sc.ny, sc.nz, sc.dx, sc.dt, sc.nsteps, sc.npml, sc.lam, sc.mu, sc.rho,
                   sc.alpha, sc.rec, precision=precision, **kw)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.el_plan_destroy(h)   # the library handle outlives module teardown
        self._h = None

    __del__ = close

    # ----------------------------------------------------------- operators
    def forward(self, p0, out=None, stream=None) -> torch.Tensor:
        """traces[M][L] (float64, device) = H p0."""
        p = torch.as_tensor(p0).to(device=self.device, dtype=self.dtype).contiguous()
        assert p.numel() == self.N
        if out is None:
            out = torch.empty((self.nsteps, self.nrec), dtype=torch.float64, device=self.device)
        assert out.dtype == torch.float64 and out.is_contiguous() and out.numel() == self.nsteps * self.nrec
        with torch.cuda.device(self.device):
            _check(lib().el_forward(self._h, ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    _stream(stream)))
        return out

    def forward_energy(self, p0, every: int = 1, out=None, stream=None):
        """(traces, energy): traces = H p0 as forward(), and the modified energy E_m (float64,
        device) of the time levels m = 0, every, ... <= M - 2 (el_forward_energy)."""
        p = torch.as_tensor(p0).to(device=self.device, dtype=self.dtype).contiguous()
        assert p.numel() == self.N
        if out is None:
            out = torch.empty((self.nsteps, self.nrec), dtype=torch.float64, device=self.device)
        assert out.dtype == torch.float64 and out.is_contiguous() and out.numel() == self.nsteps * self.nrec
        every = int(every)
        ne = (self.nsteps - 1 + every - 1) // every if self.nsteps > 1 and every >= 1 else 0
        energy = torch.empty(max(ne, 1), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().el_forward_energy(self._h, ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                           every, ctypes.c_void_p(energy.data_ptr()), _stream(stream)))
        return out, energy[:ne]

    def adjoint(self, y, out=None, stream=None) -> torch.Tensor:
        """p_adj[nz][ny][nx] (plan precision, device) = H^T y."""
        yy = torch.as_tensor(y).to(device=self.device, dtype=torch.float64).contiguous()
        assert yy.numel() == self.nsteps * self.nrec
        if out is None:
            out = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        assert out.dtype == self.dtype and out.is_contiguous() and out.numel() == self.N
        with torch.cuda.device(self.device):
            _check(lib().el_adjoint(self._h, ctypes.c_void_p(yy.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    _stream(stream)))
        return out

    def dot(self, a, b, space: int, stream=None) -> torch.Tensor:
        """<a, b> in float64 on the device; space 0 = volume (plan precision), 1 = traces."""
        dt = self.dtype if space == 0 else torch.float64
        aa = torch.as_tensor(a).to(device=self.device, dtype=dt).contiguous()
        bb = torch.as_tensor(b).to(device=self.device, dtype=dt).contiguous()
        out = torch.empty((), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().el_dot_f64(self._h, int(space), ctypes.c_void_p(aa.data_ptr()),
                                    ctypes.c_void_p(bb.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    _stream(stream)))
        return out

    def fluid_path(self, enable: bool | None = None) -> tuple[int, int]:
        """Switch the fluid-tile update on or off (None keeps the setting); returns the number
        of tiles and of cells that take it (el_plan_fluid_path)."""
        st = self.fluid_stats(enable)
        return st["tiles"], st["cells"]

    def fluid_stats(self, enable: bool | None = None) -> dict:
        """As fluid_path, returning every count of el_fluid_stats: tiles, cells, layer_cells
        (fluid cells in C-PML layers summed over the three axes), skipped_stores (s22 / s33
        stores one stress pass leaves out), uniform_cells (fluid cells whose lambda, rho
        and alpha come from the per-tile table) and column_cells (cells of fluid columns
        inside tiles that are not fluid; counted in cells too)."""
        st = FluidStats()
        flag = -1 if enable is None else (1 if enable else 0)
        _check(lib().el_plan_fluid_path(self._h, flag, ctypes.byref(st)))
        return {name: int(getattr(st, name)) for name, _ in FluidStats._fields_}

    def relaxation_extent(self) -> tuple[int, int, int]:
        """(tiles, cells, points): the tiles the relaxation sub-update visits, their cells, and
        the (cell, component) velocity points it updates (el_plan_relaxation)."""
        t, c, p = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
        _check(lib().el_plan_relaxation(self._h, ctypes.byref(t), ctypes.byref(c), ctypes.byref(p)))
        return int(t.value), int(c.value), int(p.value)

    def timing(self, enable: bool = True, every: int = 1):
        """Record an event pair around the time-loop kernel launches of every `every`-th time
        step of later operations (el_plan_timing); enable=False stops recording."""
        _check(lib().el_plan_timing(self._h, int(every) if enable else 0))

    def kernel_times(self) -> dict:
        """{kernel: (launches, total_ms)} recorded since the last call (host-blocking)."""
        out = {}
        for k, name in enumerate(KERNELS):
            n = ctypes.c_int64(0)
            ms = ctypes.c_double(0.0)
            _check(lib().el_plan_kernel_time(self._h, k, ctypes.byref(n), ctypes.byref(ms)))
            out[name] = (int(n.value), float(ms.value))
        return out

    def field(self, name) -> torch.Tensor:
        """View of one of the plan's wavefield arrays (u1..s12) inside the workspace."""
        fid = FIELDS.index(name) if isinstance(name, str) else int(name)
        ptr = ctypes.c_void_p(None)
        cnt = ctypes.c_size_t(0)
        _check(lib().el_plan_field(self._h, fid, ctypes.byref(ptr), ctypes.byref(cnt)))
        px, pl, org = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
        _check(lib().el_plan_layout(self._h, ctypes.byref(px), ctypes.byref(pl), ctypes.byref(org)))
        off = ptr.value - self.workspace.data_ptr()
        es = 8 if self.precision == "f64" else 4
        flat = self.workspace[off:off + cnt.value * es].view(self.dtype)
        nz, ny, nx = self.shape
        return flat.as_strided((nz, ny, nx), (pl.value, px.value, 1), flat.storage_offset() + org.value)


def dot_noalloc(a: torch.Tensor, b: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """<a, b> in float64 on the device without a plan or device allocation by the library
    (el_dot_f64_noalloc); a, b are contiguous float32 or float64 device tensors of equal size."""
    if a.dtype != b.dtype or a.dtype not in (torch.float32, torch.float64) or a.numel() != b.numel():
        raise ValueError("a and b must be float32 or float64 tensors of one dtype and size")
    if not (a.is_cuda and b.is_cuda and a.is_contiguous() and b.is_contiguous()):
        raise ValueError("a and b must be contiguous device tensors")
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=a.device)
    prec = EL_F64 if a.dtype == torch.float64 else EL_F32
    _check(lib().el_dot_f64_noalloc(prec, a.numel(), ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                    ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def eir_apply(h: torch.Tensor, traces: torch.Tensor, transpose: bool = False, out=None, stream=None) -> torch.Tensor:
    """Convolve every trace (float64 [M][L] on the device) in time with the causal kernel h
    (el_eir_apply), or correlate with it when transpose is set (the adjoint)."""
    if traces.dim() != 2 or traces.dtype != torch.float64 or not traces.is_cuda:
        raise ValueError("traces must be a float64 [M][L] device tensor")
    traces = traces.contiguous()
    hd = h.to(device=traces.device, dtype=torch.float64).contiguous()
    if out is None:
        out = torch.empty_like(traces)
    M, L = traces.shape
    _check(lib().el_eir_apply(hd.data_ptr(), hd.numel(), traces.data_ptr(), out.data_ptr(), M, L,
                              1 if transpose else 0, _stream(stream)))
    return out


class WithResponse:
    """The imaging model with a transducer response: forward E H p, adjoint H^T E^T y
    (E = el_eir_apply with kernel h).  Has the forward/adjoint/shape/dtype/device interface
    of a Plan, so the reconstruction solvers accept it."""

    def __init__(self, plan: "Plan", h: torch.Tensor):
        self.plan = plan
        self.h = h.to(device=plan.device, dtype=torch.float64).contiguous()
        self.shape, self.dtype, self.device = plan.shape, plan.dtype, plan.device

    def forward(self, p0):
        return eir_apply(self.h, self.plan.forward(p0))

    def adjoint(self, y):
        return self.plan.adjoint(eir_apply(self.h, y.to(torch.float64), transpose=True))


class Executor:
    """Several operator applications in flight at once (one HIP stream per slot).

    start() enqueues a whole forward or adjoint application of a plan on a free
    slot and returns the slot; poll()/wait() report completion.  The plan and
    the in/out tensors are kept alive here until the operation has completed.
    With ahead > 0 each slot keeps at most that many graph replays in flight and
    poll()/pump()/wait() enqueue the rest as earlier ones finish.
    """

    def __init__(self, max_slots: int = 4, chunk: int = 64, device=None, ahead: int = 0):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        h = ctypes.c_void_p(None)
        with torch.cuda.device(self.device):
            _check(lib().el_exec_create(ctypes.byref(h), int(max_slots), int(chunk)))
        self._h = h
        self._lib = lib()
        self.max_slots = int(max_slots)
        self._held = {}
        if ahead:
            self.set_ahead(ahead)

    def set_ahead(self, replays: int):
        with torch.cuda.device(self.device):
            _check(lib().el_exec_set_ahead(self._h, int(replays)))
        self.ahead = int(replays)

    def pump(self):
        """Enqueue what the replay limit allows on every running slot."""
        with torch.cuda.device(self.device):
            _check(lib().el_exec_pump(self._h))

    def start(self, plan: "Plan", op: int, inp: torch.Tensor, out: torch.Tensor, stream=None) -> int:
        """The operation is ordered after the work enqueued so far on `stream` (default: the
        current torch stream, which wrote inp)."""
        slot = ctypes.c_int32(-1)
        with torch.cuda.device(self.device):
            _check(lib().el_exec_start(self._h, plan._h, int(op), ctypes.c_void_p(inp.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), _stream(stream), ctypes.byref(slot)))
        self._held[slot.value] = (plan, inp, out)
        return slot.value

    def poll(self, slot: int) -> bool:
        done = ctypes.c_int32(0)
        with torch.cuda.device(self.device):
            _check(lib().el_exec_poll(self._h, int(slot), ctypes.byref(done)))
        if done.value:
            self._held.pop(slot, None)
        return bool(done.value)

    def wait(self, slot: int):
        with torch.cuda.device(self.device):
            _check(lib().el_exec_wait(self._h, int(slot)))
        self._held.pop(slot, None)

    def slots(self):
        t, b = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().el_exec_slots(self._h, ctypes.byref(t), ctypes.byref(b)))
        return t.value, b.value

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            if torch is not None and torch.cuda is not None:
                with torch.cuda.device(self.device):
                    self._lib.el_exec_destroy(h)   # the library handle outlives module teardown
            else:
                self._lib.el_exec_destroy(h)
        self._h = None
        self._held = {}

    __del__ = close


class Group:
    """Grouped time stepping of many operator applications (el_group).

    add() makes a forward or adjoint application of a plan a member; run(ticks)
    advances every running member by `ticks` time steps, up to four members per
    launch; poll() reports a member's completion; remove() withdraws one.  The
    plans and in/out tensors are kept alive here until their member is done.
    """

    def __init__(self, max_members: int = 8, precision: int = EL_F32, device=None):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        h = ctypes.c_void_p(None)
        with torch.cuda.device(self.device):
            _check(lib().el_group_create(ctypes.byref(h), int(max_members), int(precision)))
        self._h = h
        self._lib = lib()
        self.max_members = int(max_members)
        self._held = {}

    def add(self, plan: "Plan", op: int, inp: torch.Tensor, out: torch.Tensor, stream=None) -> int:
        """The member starts after the work enqueued so far on `stream` (default: the current
        torch stream, which wrote inp)."""
        slot = ctypes.c_int32(-1)
        with torch.cuda.device(self.device):
            _check(lib().el_group_add(self._h, plan._h, int(op), ctypes.c_void_p(inp.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), _stream(stream), ctypes.byref(slot)))
        self._held[slot.value] = (plan, inp, out)
        return slot.value

    def run(self, ticks: int):
        with torch.cuda.device(self.device):
            _check(lib().el_group_run(self._h, int(ticks)))

    def sync(self, pending: int = 0):
        with torch.cuda.device(self.device):
            _check(lib().el_group_sync(self._h, int(pending)))

    def poll(self, slot: int):
        """(steps enqueued, done)."""
        steps, done = ctypes.c_int32(0), ctypes.c_int32(0)
        with torch.cuda.device(self.device):
            _check(lib().el_group_poll(self._h, int(slot), ctypes.byref(steps), ctypes.byref(done)))
        if done.value:
            self._held.pop(slot, None)
        return steps.value, bool(done.value)

    def remove(self, slot: int):
        with torch.cuda.device(self.device):
            _check(lib().el_group_remove(self._h, int(slot)))

    def members(self):
        """(slots, slots in use, members still stepping)."""
        t, u, r = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().el_group_members(self._h, ctypes.byref(t), ctypes.byref(u), ctypes.byref(r)))
        return t.value, u.value, r.value

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            if torch is not None and torch.cuda is not None:
                with torch.cuda.device(self.device):
                    self._lib.el_group_destroy(h)
            else:
                self._lib.el_group_destroy(h)
        self._h = None
        self._held = {}

    __del__ = close
