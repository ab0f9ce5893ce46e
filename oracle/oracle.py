"""Python access to the FP64 CPU oracle of the MRTLB-VANSE time step.

TEST INFRASTRUCTURE.  The oracle (``vanse_oracle.c``) is the plain, literal
reference that the GPU path is checked against: whole-field passes in the
order of Sec. 2.3 of Liu, Zhang, Min & Wu (arXiv:2409.02964), the matrices of
Eq. (A1) applied as written, push streaming.  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark import this module; the
product package never does, and this module imports nothing from it.

Fields are numpy float64 arrays of shape (ny, nx); populations (9, ny, nx).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vanse_oracle.c")
_LIB = os.path.join(_HERE, "libvanse_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O3 without fast-math, no FMA contraction,
    OpenMP over nodes (thread count from OMP_NUM_THREADS)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O3", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
            "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("bc_x", C.c_int),
                ("bc_y", C.c_int), ("kappa", C.c_double), ("s_c", C.c_double),
                ("s_e", C.c_double), ("s_eps", C.c_double), ("s_q", C.c_double),
                ("s_nu", C.c_double), ("gx", C.c_double), ("gy", C.c_double),
                ("scale_by_phi", C.c_int), ("use_penalty", C.c_int),
                ("beta", C.POINTER(C.c_double)), ("usx", C.c_double), ("usy", C.c_double),
                ("model_b", C.c_int), ("eq2", C.c_int), ("uw_lo", C.c_double),
                ("uw_hi", C.c_double), ("rho_w", C.c_double),
                ("nee_lo", C.c_int), ("nee_hi", C.c_int), ("un_lo", C.c_double),
                ("un_hi", C.c_double)]


_D = C.POINTER(C.c_double)
_U8 = C.POINTER(C.c_ubyte)


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=False)
            L = C.CDLL(_LIB)
            P = C.POINTER(_Params)
            L.vo_tables.argtypes = [_D, _D, C.POINTER(C.c_int), C.POINTER(C.c_int), _D,
                                    C.POINTER(C.c_int)]
            L.vo_feq.argtypes = [C.c_double] * 5 + [_D]
            L.vo_meq.argtypes = [C.c_double] * 5 + [_D]
            L.vo_feq2.argtypes = [C.c_double] * 5 + [_D]
            L.vo_meq2.argtypes = [C.c_double] * 5 + [_D]
            L.vo_penalty_b3.argtypes = [C.c_double] * 5 + [_D, _D]
            L.vo_force_moments.argtypes = [C.c_double] * 4 + [_D]
            L.vo_penalty.argtypes = [C.c_double] * 4 + [_D, _D]
            L.vo_gradient.argtypes = [P, _U8, _D, C.c_int, _D, _D]
            L.vo_macroscopic.argtypes = [P, _D, _U8, _D, _D, _D] + [_D] * 7
            L.vo_step.argtypes = [P, _D, _D, _U8, _D, _D, _D, _D]
            L.vo_step.restype = C.c_int
            L.vo_init_equilibrium.argtypes = [P, _D, _U8, C.c_double, C.c_double,
                                              C.c_double, _D]
            L.vo_init_fields.argtypes = [P, _D, _U8, _D, _D, _D, _D]
            L.vo_run.argtypes = [P, _D, _U8, _D, _D, _D, C.c_long]
            L.vo_run.restype = C.c_int
            L.vo_set_threads.argtypes = [C.c_int]
            L.vo_threads.restype = C.c_int
            _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = np.broadcast_to(a, shape).copy() if a.shape != shape else a
    return a


def set_threads(n: int) -> int:
    """Use n OpenMP threads for the per-node loops; returns the count in use."""
    lib().vo_set_threads(int(n))
    return lib().vo_threads()


def tables():
    """The constants the oracle uses: M, 36*M^-1 (Eq. A1), e_i, w_i, opposite."""
    M = np.zeros(81)
    Mi = np.zeros(81)
    ex = (C.c_int * 9)()
    ey = (C.c_int * 9)()
    w = np.zeros(9)
    opp = (C.c_int * 9)()
    lib().vo_tables(_dp(M), _dp(Mi), ex, ey, _dp(w), opp)
    return (M.reshape(9, 9), Mi.reshape(9, 9), np.array(list(ex)), np.array(list(ey)),
            w, np.array(list(opp)))


def feq(phi, rho, ux, uy, kappa):
    out = np.zeros(9)
    lib().vo_feq(phi, rho, ux, uy, kappa, _dp(out))
    return out


def meq(phi, rho, ux, uy, kappa):
    out = np.zeros(9)
    lib().vo_meq(phi, rho, ux, uy, kappa, _dp(out))
    return out


def feq2(phi, rho, ux, uy, kappa):
    out = np.zeros(9)
    lib().vo_feq2(phi, rho, ux, uy, kappa, _dp(out))
    return out


def meq2(phi, rho, ux, uy, kappa):
    out = np.zeros(9)
    lib().vo_meq2(phi, rho, ux, uy, kappa, _dp(out))
    return out


def force_moments(ux, uy, Fx, Fy):
    out = np.zeros(9)
    lib().vo_force_moments(ux, uy, Fx, Fy, _dp(out))
    return out


def penalty(phi, rho, kappa, dt_phi, d8):
    d8 = _f64(d8)
    out = np.zeros(3)
    lib().vo_penalty(phi, rho, kappa, dt_phi, _dp(d8), _dp(out))
    return out


def penalty_b3(phi, rho, kappa, kmp, dt_phi, d12):
    d12 = _f64(d12)
    out = np.zeros(3)
    lib().vo_penalty_b3(phi, rho, kappa, kmp, dt_phi, _dp(d12), _dp(out))
    return out


BC = {"periodic": 0, "wall": 1}


class Oracle:
    """One lattice stepped by the oracle.

    ``rates`` are the diagonal entries of Gamma (Eq. 16) -- the paper's tau_*
    read as relaxation rates: dict with keys s_c, s_e, s_eps, s_q, s_nu.
    """

    def __init__(self, nx, ny, phi, kappa=0.5, rates=None, g=(0.0, 0.0),
                 scale_by_phi=True, bc_x="periodic", bc_y="periodic", mask=None,
                 force=None, penalty=True, drag=None, model_b=False, eq2=False,
                 wall_velocity=(0.0, 0.0), rho_w=1.0, velocity_rows=(None, None)):
        r = dict(s_c=1.0, s_e=1.2, s_eps=1.2, s_q=1.2, s_nu=1.2)
        if rates:
            r.update(rates)
        self.nx, self.ny = int(nx), int(ny)
        self.p = _Params(self.nx, self.ny, BC[bc_x], BC[bc_y], float(kappa), r["s_c"],
                         r["s_e"], r["s_eps"], r["s_q"], r["s_nu"], float(g[0]),
                         float(g[1]), 1 if scale_by_phi else 0, 1 if penalty else 0)
        self.p.model_b = 1 if model_b else 0
        self.p.eq2 = 1 if eq2 else 0
        # x velocities of the walls at y = -1/2 and y = ny - 1/2 (bc_y = "wall")
        self.p.uw_lo, self.p.uw_hi = float(wall_velocity[0]), float(wall_velocity[1])
        self.p.rho_w = float(rho_w)
        # velocity boundary rows (non-equilibrium extrapolation, Sec. 3.1):
        # x velocity of the first / last row, None for an ordinary row
        lo, hi = velocity_rows
        if (lo is not None or hi is not None) and bc_y != "wall":
            raise ValueError("velocity rows need walls in y")
        self.p.nee_lo, self.p.un_lo = (0, 0.0) if lo is None else (1, float(lo))
        self.p.nee_hi, self.p.un_hi = (0, 0.0) if hi is None else (1, float(hi))
        self.velocity_rows = velocity_rows
        shp = (self.ny, self.nx)
        self.phi = _f64(phi, shp)
        if drag is not None:  # (beta field, (usx, usy)): F^B -= phi beta (u - u_s)
            self.beta = _f64(drag[0], shp)
            self.p.beta = _dp(self.beta)
            self.p.usx, self.p.usy = float(drag[1][0]), float(drag[1][1])
        self.mask = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        if force is None:
            self.fx = self.fy = None
        else:
            self.fx = _f64(force[0], shp)
            self.fy = _f64(force[1], shp)
        self.f = np.zeros((9,) + shp)
        self.t = 0

    def _mask(self):
        return None if self.mask is None else self.mask.ctypes.data_as(_U8)

    def init_equilibrium(self, rho0=1.0, ux0=0.0, uy0=0.0):
        lib().vo_init_equilibrium(C.byref(self.p), _dp(self.phi), self._mask(), rho0, ux0,
                                  uy0, _dp(self.f))
        self.t = 0
        return self

    def init_fields(self, rho, ux, uy):
        shp = (self.ny, self.nx)
        rho, ux, uy = _f64(rho, shp), _f64(ux, shp), _f64(uy, shp)
        lib().vo_init_fields(C.byref(self.p), _dp(self.phi), self._mask(), _dp(rho),
                             _dp(ux), _dp(uy), _dp(self.f))
        self.t = 0
        return self

    def set_populations(self, f):
        self.f = _f64(f, (9, self.ny, self.nx)).copy()

    def step(self, n=1, phi_next=None):
        """Advance n steps.  With ``phi_next`` (only for n == 1) the d_t phi
        term of Eq. (20) uses it and phi becomes phi_next afterwards."""
        if phi_next is not None:
            assert n == 1
            pn = _f64(phi_next, (self.ny, self.nx))
            out = np.empty_like(self.f)
            rc = lib().vo_step(C.byref(self.p), _dp(self.phi), _dp(pn), self._mask(),
                               _dp(self.fx), _dp(self.fy), _dp(self.f), _dp(out))
            if rc != 0:
                raise MemoryError("oracle step failed")
            self.f = out
            self.phi = pn
            self.t += 1
            return self
        rc = lib().vo_run(C.byref(self.p), _dp(self.phi), self._mask(), _dp(self.fx),
                          _dp(self.fy), _dp(self.f), int(n))
        if rc != 0:
            raise MemoryError("oracle run failed")
        self.t += int(n)
        return self

    def macroscopic(self):
        """dict of m0 (= sum f = phi*rho), rho, ux, uy, Fx, Fy, p (Eq. 7, 13)."""
        shp = (self.ny, self.nx)
        out = {k: np.zeros(shp) for k in ("m0", "rho", "ux", "uy", "Fx", "Fy", "p")}
        lib().vo_macroscopic(C.byref(self.p), _dp(self.phi), self._mask(), _dp(self.fx),
                             _dp(self.fy), _dp(self.f), *[_dp(out[k]) for k in
                                                           ("m0", "rho", "ux", "uy", "Fx",
                                                            "Fy", "p")])
        return out

    def gradient(self, psi, odd=False):
        psi = _f64(psi, (self.ny, self.nx))
        gx = np.zeros_like(psi)
        gy = np.zeros_like(psi)
        lib().vo_gradient(C.byref(self.p), self._mask(), _dp(psi), 1 if odd else 0,
                          _dp(gx), _dp(gy))
        return gx, gy

    def fluid(self):
        """Boolean (ny, nx) map of the fluid nodes: not solid and not on a
        velocity boundary row."""
        m = np.ones((self.ny, self.nx), bool) if self.mask is None else self.mask == 0
        m = m.copy()
        if self.p.nee_lo:
            m[0] = False
        if self.p.nee_hi:
            m[-1] = False
        return m

    def mass(self):
        """Total mass: exactly rounded sum over fluid nodes of sum_i f_i."""
        import math
        return math.fsum(self.f[:, self.fluid()].ravel().tolist())
