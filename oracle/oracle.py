"""ctypes front end of the FP64 CPU oracle (el_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the operator library or its
Python binding.  It shares no code with the GPU path.

Functions follow the paper's discrete operators (Mitsuhashi et al., Sec. 3-4
and the Appendix "Discrete formulation"):
  forward(p0)   -> traces [M][L] = H p0           (eq. HPML)
  adjoint(y)    -> p [N]         = H^T y          (eq. adjHPML, recursion eq. AdjupPML)
  step(v, tr)   -> v <- W' v  or  W'^T v          (27N state, Appendix)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "el_oracle.c")
_LIB = os.path.join(_HERE, "libel_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile el_oracle.c with gcc (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dt", ctypes.c_double),
                ("nsteps", ctypes.c_int32), ("npml", ctypes.c_int32),
                ("pml_R", ctypes.c_double), ("pml_npower", ctypes.c_double), ("pml_f0", ctypes.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        L.eo_model_create.restype = vp
        L.eo_model_create.argtypes = [ctypes.POINTER(_Grid), vp, vp, vp, vp, vp, ctypes.c_int32]
        L.eo_model_free.argtypes = [vp]
        L.eo_ncells.restype = ctypes.c_int64
        L.eo_ncells.argtypes = [vp]
        L.eo_cmax.restype = ctypes.c_double
        L.eo_cmax.argtypes = [vp]
        L.eo_coefficients.argtypes = [vp, vp, vp, vp, vp, vp]
        L.eo_pml_table.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]
        L.eo_receivers.argtypes = [vp, vp, vp]
        L.eo_step.argtypes = [vp, vp, ctypes.c_int]
        L.eo_inject.argtypes = [vp, vp, vp]
        L.eo_extract.argtypes = [vp, vp, vp]
        L.eo_measure.argtypes = [vp, vp, vp]
        L.eo_measure_tr.argtypes = [vp, vp, vp]
        L.eo_forward.restype = ctypes.c_int
        L.eo_forward.argtypes = [vp, vp, vp, ctypes.c_int32]
        L.eo_adjoint.restype = ctypes.c_int
        L.eo_adjoint.argtypes = [vp, vp, vp, ctypes.c_int32]
        L.eo_run.argtypes = [vp, vp, ctypes.c_int32]
        L.eo_num_threads.restype = ctypes.c_int
        L.eo_set_relaxation.restype = ctypes.c_int
        L.eo_set_relaxation.argtypes = [vp, ctypes.c_int32, vp, vp, vp]
        L.eo_state_len.restype = ctypes.c_int64
        L.eo_state_len.argtypes = [vp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Model:
    """Oracle model of one grid, medium and receiver set.

    Parameters mirror the operator library's plan: cell maps lambda, mu,
    rho, alpha (float32, [nz][ny][nx]); receivers in metres (float64 [L][3]).
    """

    def __init__(self, nx, ny, nz, dx, dt, nsteps, npml, lam, mu, rho, alpha, rec,
                 pml_R=0.0, pml_npower=0.0, pml_f0=0.0, alpha_r=None, mechanisms=None):
        """alpha_r, mechanisms: frequency-dependent absorption (el_oracle.c, eo_set_relaxation):
        the cell map of the relaxation strength (1/s) and a list of (omega_l, w_l) pairs."""
        L = lib()
        self.shape = (nz, ny, nx)
        self.nsteps = int(nsteps)
        self.g = _Grid(nx, ny, nz, dx, dt, nsteps, npml, pml_R, pml_npower, pml_f0)
        self._keep = [_f32(lam), _f32(mu), _f32(rho), _f32(alpha)]
        rec = _f64(np.asarray(rec).reshape(-1, 3)) if rec is not None else np.zeros((0, 3))
        self.nrec = rec.shape[0]
        self._rec = rec
        h = L.eo_model_create(ctypes.byref(self.g), *[_ptr(a) for a in self._keep], _ptr(rec), self.nrec)
        if not h:
            raise ValueError("oracle: invalid grid, medium or receiver outside the grid")
        self._h = ctypes.c_void_p(h)
        self.N = int(L.eo_ncells(self._h))
        self.nmech = 0
        if mechanisms:
            om = _f64([m[0] for m in mechanisms])
            wt = _f64([m[1] for m in mechanisms])
            ar = _f32(alpha_r).reshape(-1)
            assert ar.size == self.N
            if L.eo_set_relaxation(self._h, len(mechanisms), _ptr(om), _ptr(wt), _ptr(ar)) != 0:
                raise ValueError("oracle: invalid relaxation mechanisms or strength map")
            self.nmech = len(mechanisms)
        self.state_len = int(L.eo_state_len(self._h))

    @classmethod
    def from_scenario(cls, sc, **over):
        kw = dict(nx=sc.nx, ny=sc.ny, nz=sc.nz, dx=sc.dx, dt=sc.dt, nsteps=sc.nsteps,
                  npml=sc.npml, lam=sc.lam, mu=sc.mu, rho=sc.rho, alpha=sc.alpha, rec=sc.rec)
        if getattr(sc, "mechanisms", None):
            kw.update(alpha_r=sc.alpha_r, mechanisms=sc.mechanisms)
        kw.update(over)
        return cls(**kw)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.eo_model_free(h)
            self._h = None

    # -------------------------------------------------------------- operators
    def forward(self, p0, nsteps: int = 0) -> np.ndarray:
        M = nsteps or self.nsteps
        p = _f64(p0).reshape(-1)
        assert p.size == self.N
        out = np.zeros((M, self.nrec), dtype=np.float64)
        rc = lib().eo_forward(self._h, _ptr(p), _ptr(out), M)
        if rc != 0:
            raise MemoryError("oracle forward failed")
        return out

    def adjoint(self, y, nsteps: int = 0) -> np.ndarray:
        M = nsteps or self.nsteps
        yy = _f64(y).reshape(M, self.nrec)
        out = np.zeros(self.N, dtype=np.float64)
        rc = lib().eo_adjoint(self._h, _ptr(yy), _ptr(out), M)
        if rc != 0:
            raise MemoryError("oracle adjoint failed")
        return out.reshape(self.shape)

    def step(self, v: np.ndarray, transpose: bool = False) -> np.ndarray:
        """v <- W' v (or W'^T v) in place on a float64 state of state_len entries (27N, plus
        3N per relaxation mechanism)."""
        assert v.dtype == np.float64 and v.flags.c_contiguous and v.size == self.state_len
        lib().eo_step(self._h, _ptr(v), 1 if transpose else 0)
        return v

    def run(self, v: np.ndarray, steps: int) -> np.ndarray:
        assert v.dtype == np.float64 and v.flags.c_contiguous and v.size == self.state_len
        lib().eo_run(self._h, _ptr(v), int(steps))
        return v

    def inject(self, p0) -> np.ndarray:
        v = np.zeros(self.state_len)
        p = _f64(p0).reshape(-1)
        lib().eo_inject(self._h, _ptr(p), _ptr(v))
        return v

    def extract(self, v) -> np.ndarray:
        out = np.zeros(self.N)
        lib().eo_extract(self._h, _ptr(v), _ptr(out))
        return out

    def measure(self, v) -> np.ndarray:
        out = np.zeros(self.nrec)
        lib().eo_measure(self._h, _ptr(v), _ptr(out))
        return out

    def measure_tr(self, y, v) -> np.ndarray:
        yy = _f64(y)
        lib().eo_measure_tr(self._h, _ptr(yy), _ptr(v))
        return v

    # ------------------------------------------------------------ inspection
    def coefficients(self) -> dict:
        N = self.N
        rho_u = np.zeros(3 * N); alpha_u = np.zeros(3 * N); lam = np.zeros(N); mu = np.zeros(N)
        mu_s = np.zeros(3 * N)
        lib().eo_coefficients(self._h, _ptr(rho_u), _ptr(alpha_u), _ptr(lam), _ptr(mu), _ptr(mu_s))
        sh = self.shape
        return dict(rho_u=rho_u.reshape((3,) + sh), alpha_u=alpha_u.reshape((3,) + sh),
                    lam=lam.reshape(sh), mu=mu.reshape(sh), mu_s=mu_s.reshape((3,) + sh))

    def pml_table(self, axis: int, half: int):
        n = (self.g.nx, self.g.ny, self.g.nz)[axis]
        a = np.zeros(n); b = np.zeros(n); chi = np.zeros(n)
        lib().eo_pml_table(self._h, axis, half, _ptr(a), _ptr(b), _ptr(chi))
        return a, b, chi

    def receivers(self):
        base = np.zeros((self.nrec, 8), dtype=np.int64)
        w = np.zeros((self.nrec, 8))
        if self.nrec:
            lib().eo_receivers(self._h, _ptr(base), _ptr(w))
        return base, w

    @property
    def cmax(self) -> float:
        return float(lib().eo_cmax(self._h))

    # ------------------------------------------------------------ state views
    def state_views(self, v: np.ndarray) -> dict:
        """Named views of a state: phi[3][3], u[3], psi[3][3], sig[6] (Voigt order) and the
        relaxation memory variables zeta[l][3]."""
        N, sh = self.N, self.shape
        f = lambda k: v[k * N:(k + 1) * N].reshape(sh)
        return dict(phi=[[f(3 * i + j) for j in range(3)] for i in range(3)],
                    u=[f(9 + i) for i in range(3)],
                    psi=[[f(12 + 3 * i + j) for j in range(3)] for i in range(3)],
                    sig=[f(21 + a) for a in range(6)],
                    zeta=[[f(27 + 3 * l + i) for i in range(3)] for l in range(self.nmech)])


def num_threads() -> int:
    return int(lib().eo_num_threads())


if __name__ == "__main__":
    print(build(force=True), file=sys.stderr)
