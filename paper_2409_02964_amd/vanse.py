"""Python binding of libvanse (the C ABI in include/vanse.h).

Argument marshalling only: torch supplies the device workspace, the field
tensors and the stream; every step of the method runs in the library's HIP
kernels.  If ``libvanse.so`` is missing or cannot be loaded, every entry point
raises -- there is no fallback path.

    lat = Lattice(4096, 4096, precision="f32", bc_y="wall")
    lat.set_params(kappa=0.5, rates=dict(s_nu=0.8, s_e=1.2, s_eps=1.2, s_q=1.2))
    lat.set_void_fraction(phi)              # (ny, nx) float64, any device
    lat.set_body_force(1e-7, 0.0)
    lat.init_equilibrium(rho0=1.0)
    lat.step(10000)
    m = lat.read_moments()                  # dict of (ny, nx) float64 cuda tensors
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvanse.so")

PRECISION = {"f64": 0, "f32": 1, "f32s": 2, "f16s": 3}
BC = {"periodic": 0, "wall": 1}
ERRORS = {0: "ok", -1: "invalid argument", -2: "workspace", -3: "HIP error", -4: "state",
          -5: "diverged", -6: "unsupported"}

EXPORTS = [
    "vanse_workspace_bytes", "vanse_create", "vanse_destroy", "vanse_set_params",
    "vanse_set_scheme", "vanse_set_wall_velocity", "vanse_set_velocity_rows",
    "vanse_set_body_force",
    "vanse_set_void_fraction",
    "vanse_set_void_fraction_next",
    "vanse_set_void_fraction_next2",
    "vanse_set_mask", "vanse_set_force_field", "vanse_set_drag",
    "vanse_init_equilibrium", "vanse_set_populations", "vanse_step",
    "vanse_set_check_interval", "vanse_read_moments",
    "vanse_read_populations", "vanse_observe", "vanse_observe_noalloc", "vanse_residual",
    "vanse_set_tiling",
    "vanse_get_tiling", "vanse_set_steps_per_pass", "vanse_get_fused_tiling",
    "vanse_set_storage_exponent", "vanse_stream_copy", "vanse_time", "vanse_error_string",
    "vanse_last_error", "vanse_batch_workspace_bytes", "vanse_batch_create", "vanse_batch_destroy",
    "vanse_batch_workspace_bytes_ex", "vanse_batch_create_ex",
    "vanse_batch_set_graph", "vanse_batch_step", "vanse_batch_residual", "vanse_batch_tiles",
]


class VanseError(RuntimeError):
    def __init__(self, code, detail):
        super().__init__(f"{ERRORS.get(code, code)} ({code}): {detail}")
        self.code = code


class Diverged(VanseError):
    pass


class Desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("precision", C.c_int32),
                ("bc_x", C.c_int32), ("bc_y", C.c_int32), ("has_force_field", C.c_int32),
                ("has_drag", C.c_int32), ("has_mask", C.c_int32), ("dynamic_phi", C.c_int32)]


class Rates(C.Structure):
    _fields_ = [("s_c", C.c_double), ("s_e", C.c_double), ("s_eps", C.c_double),
                ("s_q", C.c_double), ("s_nu", C.c_double)]


_lock = threading.Lock()
_lib = None


def lib():
    """Load libvanse.so (raises if it is not built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
            L = C.CDLL(LIB_PATH)
            vp, d, i32, i64 = C.c_void_p, C.c_double, C.c_int, C.c_int64
            pd = C.POINTER(C.c_double)
            sig = {
                "vanse_workspace_bytes": [C.POINTER(Desc), C.POINTER(C.c_size_t)],
                "vanse_create": [C.POINTER(Desc), vp, C.c_size_t, C.POINTER(vp)],
                "vanse_destroy": [vp],
                "vanse_set_params": [vp, d, C.POINTER(Rates)],
                "vanse_set_body_force": [vp, d, d, i32],
                "vanse_set_scheme": [vp, i32, i32],
                "vanse_set_wall_velocity": [vp, d, d],
                "vanse_set_velocity_rows": [vp, i32, d, d],
                "vanse_set_void_fraction": [vp, vp, vp],
                "vanse_set_void_fraction_next": [vp, vp, vp],
                "vanse_set_void_fraction_next2": [vp, vp, vp, vp, vp, vp, vp],
                "vanse_set_mask": [vp, vp, vp],
                "vanse_set_force_field": [vp, vp, vp, vp],
                "vanse_set_drag": [vp, vp, d, d, vp],
                "vanse_init_equilibrium": [vp, d, d, d, vp],
                "vanse_set_populations": [vp, vp, d, vp],
                "vanse_step": [vp, i64, vp],
                "vanse_set_check_interval": [vp, i64],
                "vanse_read_moments": [vp, vp, vp, vp, vp, vp],
                "vanse_read_populations": [vp, vp, vp],
                "vanse_observe": [vp, pd, vp],
                "vanse_observe_noalloc": [vp, pd, vp],
                "vanse_residual": [vp, pd, vp],
                "vanse_set_tiling": [vp, i32, i32],
                "vanse_get_tiling": [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)],
                "vanse_set_steps_per_pass": [vp, i32, i32],
                "vanse_get_fused_tiling": [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)],
                "vanse_set_storage_exponent": [vp, i32],
                "vanse_stream_copy": [vp, i64, vp],
                "vanse_time": [vp],
                "vanse_batch_workspace_bytes": [C.POINTER(vp), i32, i32, i32,
                                                C.POINTER(C.c_size_t)],
                "vanse_batch_create": [C.POINTER(vp), i32, i32, i32, vp, C.c_size_t,
                                       C.POINTER(vp)],
                "vanse_batch_workspace_bytes_ex": [C.POINTER(vp), i32, i32, i32, i32,
                                                   C.POINTER(C.c_size_t)],
                "vanse_batch_create_ex": [C.POINTER(vp), i32, i32, i32, i32, vp, C.c_size_t,
                                          C.POINTER(vp)],
                "vanse_batch_destroy": [vp],
                "vanse_batch_set_graph": [vp, i32],
                "vanse_batch_step": [vp, i64, vp],
                "vanse_batch_residual": [vp, pd, vp],
                "vanse_batch_tiles": [vp, C.POINTER(i32), C.POINTER(i32)],
                "vanse_error_string": [i32],
                "vanse_last_error": [],
            }
            for name, args in sig.items():
                fn = getattr(L, name)
                fn.argtypes = args
                fn.restype = C.c_int
            L.vanse_time.restype = C.c_int64
            L.vanse_error_string.restype = C.c_char_p
            L.vanse_last_error.restype = C.c_char_p
            _lib = L
    return _lib


def check(rc):
    if rc != 0:
        detail = lib().vanse_last_error().decode(errors="replace")
        raise (Diverged if rc == -5 else VanseError)(rc, detail)
    return rc


def workspace_bytes(nx, ny, precision="f64", bc_y="periodic", force_field=False,
                    drag=False, mask=False, dynamic_phi=False) -> int:
    desc = Desc(int(nx), int(ny), PRECISION[precision], 0, BC[bc_y], int(bool(force_field)),
                int(bool(drag)), int(bool(mask)), int(bool(dynamic_phi)))
    n = C.c_size_t()
    check(lib().vanse_workspace_bytes(C.byref(desc), C.byref(n)))
    return n.value


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Lattice:
    """One lattice whose device state lives in a torch-allocated workspace."""

    def __init__(self, nx, ny, precision="f64", bc_y="periodic", force_field=False,
                 device=None, workspace=None, drag=False, mask=False, dynamic_phi=False,
                 bc_x="periodic"):
        import torch
        self.nx, self.ny = int(nx), int(ny)
        self.precision = precision
        self.device = torch.device(device or "cuda")
        self.desc = Desc(self.nx, self.ny, PRECISION[precision], BC[bc_x], BC[bc_y],
                         int(bool(force_field)), int(bool(drag)), int(bool(mask)),
                         int(bool(dynamic_phi)))
        nbytes = C.c_size_t()
        check(lib().vanse_workspace_bytes(C.byref(self.desc), C.byref(nbytes)))
        if workspace is None:
            workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.workspace = workspace  # must outlive the handle
        self.handle = C.c_void_p()
        check(lib().vanse_create(C.byref(self.desc), C.c_void_p(workspace.data_ptr()),
                                 workspace.numel(), C.byref(self.handle)))

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().vanse_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- inputs ----
    def _field(self, a, shape):
        import torch
        t = torch.as_tensor(a, dtype=torch.float64).to(self.device).contiguous()
        if tuple(t.shape) != shape:
            raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
        return t

    def set_params(self, kappa=0.5, rates=None):
        r = dict(s_c=1.0, s_e=1.2, s_eps=1.2, s_q=1.2, s_nu=1.2)
        r.update(rates or {})
        rr = Rates(r["s_c"], r["s_e"], r["s_eps"], r["s_q"], r["s_nu"])
        check(lib().vanse_set_params(self.handle, float(kappa), C.byref(rr)))
        return self

    def set_scheme(self, model="A", equilibrium_order=3):
        """Model "A" (the consistent VANSE) or "B" (set I), and the
        equilibrium order 3 (Eq. 14) or 2 (Appendix B); before the populations."""
        check(lib().vanse_set_scheme(self.handle, {"A": 0, "B": 1}[model], int(equilibrium_order)))
        return self

    def set_wall_velocity(self, u_lo=0.0, u_hi=0.0):
        """x velocities of the walls at y = -1/2 and y = ny - 1/2 (before the populations)."""
        check(lib().vanse_set_wall_velocity(self.handle, float(u_lo), float(u_hi)))
        return self

    def set_velocity_rows(self, u_lo=None, u_hi=None):
        """Velocity boundary rows by non-equilibrium extrapolation (Couette
        flow, Sec. 3.1): x velocity of the first / last row, None for an
        ordinary row (before the populations); see vanse_set_velocity_rows."""
        faces = (1 if u_lo is not None else 0) | (2 if u_hi is not None else 0)
        check(lib().vanse_set_velocity_rows(self.handle, faces, float(u_lo or 0.0),
                                            float(u_hi or 0.0)))
        return self

    def set_body_force(self, gx, gy=0.0, scale_by_phi=True):
        check(lib().vanse_set_body_force(self.handle, float(gx), float(gy),
                                         1 if scale_by_phi else 0))
        return self

    def set_void_fraction(self, phi, stream=None):
        t = self._field(phi, (self.ny, self.nx))
        check(lib().vanse_set_void_fraction(self.handle, C.c_void_p(t.data_ptr()),
                                            _stream(stream)))
        return self

    def set_void_fraction_next(self, phi_next, stream=None):
        """phi(t+1) for the next (single) step; see vanse_set_void_fraction_next."""
        t = self._field(phi_next, (self.ny, self.nx))
        check(lib().vanse_set_void_fraction_next(self.handle, C.c_void_p(t.data_ptr()),
                                                 _stream(stream)))
        return self

    def set_void_fraction_next2(self, phi_next, phi_next2, beta_next=None, force_next=None, stream=None):
        """phi(t+1) and phi(t+2) for the next two steps, with the second
        step's drag coefficient and force field (fx, fy) when they change;
        see vanse_set_void_fraction_next2."""
        shape = (self.ny, self.nx)
        keep = [self._field(phi_next, shape), self._field(phi_next2, shape)]
        ptrs = [C.c_void_p(keep[0].data_ptr()), C.c_void_p(keep[1].data_ptr())]
        for f in ([beta_next] + ([None, None] if force_next is None else list(force_next))):
            if f is None:
                ptrs.append(C.c_void_p(None))
            else:
                keep.append(self._field(f, shape))
                ptrs.append(C.c_void_p(keep[-1].data_ptr()))
        check(lib().vanse_set_void_fraction_next2(self.handle, *ptrs, _stream(stream)))
        return self

    def set_mask(self, mask, stream=None):
        """Solid nodes: (ny, nx) array, nonzero = solid (before the populations)."""
        import torch
        t = torch.as_tensor(mask).to(self.device).ne(0).to(torch.uint8).contiguous()
        if tuple(t.shape) != (self.ny, self.nx):
            raise ValueError(f"expected shape {(self.ny, self.nx)}, got {tuple(t.shape)}")
        check(lib().vanse_set_mask(self.handle, C.c_void_p(t.data_ptr()), _stream(stream)))
        return self

    def set_force_field(self, fx, fy, stream=None):
        a = self._field(fx, (self.ny, self.nx))
        b = self._field(fy, (self.ny, self.nx))
        check(lib().vanse_set_force_field(self.handle, C.c_void_p(a.data_ptr()),
                                          C.c_void_p(b.data_ptr()), _stream(stream)))
        self._keep = (a, b)
        return self

    def set_drag(self, beta, us=(0.0, 0.0), stream=None):
        """F^B -= phi beta (u - u_s) with a per-node beta (ny, nx)."""
        b = self._field(beta, (self.ny, self.nx))
        check(lib().vanse_set_drag(self.handle, C.c_void_p(b.data_ptr()), float(us[0]),
                                   float(us[1]), _stream(stream)))
        self._keep_beta = b
        return self

    def init_equilibrium(self, rho0=1.0, ux0=0.0, uy0=0.0, stream=None):
        check(lib().vanse_init_equilibrium(self.handle, float(rho0), float(ux0), float(uy0),
                                           _stream(stream)))
        return self

    def set_populations(self, f, rho0=1.0, stream=None):
        t = self._field(f, (9, self.ny, self.nx))
        check(lib().vanse_set_populations(self.handle, C.c_void_p(t.data_ptr()), float(rho0),
                                          _stream(stream)))
        self._keep_f = t
        return self

    def set_tiling(self, threads=0, rows=0):
        check(lib().vanse_set_tiling(self.handle, int(threads), int(rows)))
        return self

    def tiling(self):
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        check(lib().vanse_get_tiling(self.handle, C.byref(a), C.byref(b), C.byref(c)))
        return dict(threads=a.value, rows=b.value, workgroups=c.value)

    def set_steps_per_pass(self, steps=2, rows=0):
        """Time steps per launch (1 or 2) of the step with the force field,
        the drag, solid nodes, a moving phi or a scheme variant; see vanse.h."""
        check(lib().vanse_set_steps_per_pass(self.handle, int(steps), int(rows)))
        return self

    def fused_tiling(self):
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        check(lib().vanse_get_fused_tiling(self.handle, C.byref(a), C.byref(b), C.byref(c)))
        return dict(active=bool(a.value), rows=b.value, workgroups=c.value)

    def set_storage_exponent(self, e):
        check(lib().vanse_set_storage_exponent(self.handle, int(e)))
        return self

    # ---- stepping ----
    def step(self, n=1, stream=None):
        check(lib().vanse_step(self.handle, int(n), _stream(stream)))
        return self

    def set_check_interval(self, k):
        """Run the FP64 observables inside step() at every multiple k of t and
        raise Diverged when one saw a non-finite node (0: off); see vanse.h."""
        check(lib().vanse_set_check_interval(self.handle, int(k)))
        return self

    def stream_copy(self, n=1, stream=None):
        """Speed-of-light reference: n launches of the step's memory pattern
        without arithmetic (permutes the stored state)."""
        check(lib().vanse_stream_copy(self.handle, int(n), _stream(stream)))
        return self

    @property
    def t(self):
        return int(lib().vanse_time(self.handle))

    # ---- outputs ----
    def read_moments(self, stream=None):
        import torch
        out = {k: torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
               for k in ("rho", "ux", "uy", "p")}
        check(lib().vanse_read_moments(self.handle, *[C.c_void_p(out[k].data_ptr())
                                                      for k in ("rho", "ux", "uy", "p")],
                                       _stream(stream)))
        return out

    def read_populations(self, stream=None):
        import torch
        out = torch.empty((9, self.ny, self.nx), dtype=torch.float64, device=self.device)
        check(lib().vanse_read_populations(self.handle, C.c_void_p(out.data_ptr()),
                                           _stream(stream)))
        return out

    def residual(self, stream=None):
        """(sum |u - u_prev|^2 or None on the first call, sum |u|^2, nonfinite):
        u_prev is the velocity at the previous call."""
        buf = (C.c_double * 3)()
        check(lib().vanse_residual(self.handle, buf, _stream(stream)))
        return (None if buf[0] < 0 else buf[0]), buf[1], int(buf[2])

    def observe(self, stream=None, raise_on_diverged=True, noalloc=False):
        """dict(mass, u2, umax, nonfinite) reduced in FP64 on the device;
        noalloc=True: the entry point that uses no workspace scratch and
        allocates nothing (vanse_observe_noalloc)."""
        buf = (C.c_double * 4)()
        fn = lib().vanse_observe_noalloc if noalloc else lib().vanse_observe
        rc = fn(self.handle, buf, _stream(stream))
        res = dict(mass=buf[0], u2=buf[1], umax=buf[2], nonfinite=int(buf[3]))
        if rc == -5 and not raise_on_diverged:
            return res
        check(rc)
        return res


class Batch:
    """Independent lattices advanced by one kernel launch per time step (per
    two with ``steps_per_pass=2``: the two-step kernel on every member).

    Members must share precision, boundary type and the force-field flag and
    be fully set up; they stay usable individually (read_moments, t).  With
    ``graph_steps`` > 0 step loops are captured in hipGraphs of that many
    time steps."""

    def __init__(self, lattices, threads=128, rows=0, graph_steps=0, device=None,
                 steps_per_pass=1):
        import torch
        self.lattices = list(lattices)
        n = len(self.lattices)
        self._arr = (C.c_void_p * n)(*[l.handle.value for l in self.lattices])
        nbytes = C.c_size_t()
        check(lib().vanse_batch_workspace_bytes_ex(self._arr, n, int(threads), int(rows),
                                                   int(steps_per_pass), C.byref(nbytes)))
        dev = device or self.lattices[0].device
        self.workspace = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=dev)
        self.handle = C.c_void_p()
        check(lib().vanse_batch_create_ex(self._arr, n, int(threads), int(rows),
                                          int(steps_per_pass),
                                          C.c_void_p(self.workspace.data_ptr()),
                                          self.workspace.numel(), C.byref(self.handle)))
        self.threads = int(threads)
        self.steps_per_pass = int(steps_per_pass)
        if graph_steps:
            self.set_graph(graph_steps)

    def set_graph(self, steps_per_graph):
        check(lib().vanse_batch_set_graph(self.handle, int(steps_per_graph)))
        return self

    def step(self, n=1, stream=None):
        check(lib().vanse_batch_step(self.handle, int(n), _stream(stream)))
        return self

    def residual(self, stream=None):
        """Lattice.residual() of every member with one synchronization: a
        list of (sum |u - u_prev|^2 or None, sum |u|^2, nonfinite)."""
        n = len(self.lattices)
        buf = (C.c_double * (3 * n))()
        rc = lib().vanse_batch_residual(self.handle, buf, _stream(stream))
        if rc not in (0, -5):
            check(rc)
        return [((None if buf[3 * k] < 0 else buf[3 * k]), buf[3 * k + 1], int(buf[3 * k + 2]))
                for k in range(n)]

    def tiles(self):
        a, b = C.c_int(), C.c_int()
        check(lib().vanse_batch_tiles(self.handle, C.byref(a), C.byref(b)))
        return dict(tiles=a.value, rows=b.value)

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().vanse_batch_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_batch(lattices, candidates=None, steps=20, repeats=2):
    """Pick the launch shape of a batch by timing a few steps of each
    candidate on the real batch (the members are advanced by the trials).
    Candidates are (threads, rows) or (threads, rows, steps_per_pass).
    Returns (best, timings): best as (threads, rows, steps_per_pass) with the
    rows the batch chose, timings in ms per time step."""
    import torch
    if candidates is None:
        candidates = [(t, r) for t in (64, 128, 256) for r in (0, 8, 16, 32, 64)]
    times = {}
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    for cand in candidates:
        th, rows = cand[0], cand[1]
        spp = cand[2] if len(cand) > 2 else 1
        b = Batch(lattices, threads=th, rows=rows, steps_per_pass=spp)
        b.step(2)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(repeats):
            ev0.record()
            b.step(steps)
            ev1.record()
            torch.cuda.synchronize()
            best = min(best, ev0.elapsed_time(ev1) / steps)
        times[(th, b.tiles()["rows"], spp)] = best
        b.close()
    best = min(times, key=times.get)
    return best, times
