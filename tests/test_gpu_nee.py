"""GPU parity of the velocity boundary rows (Couette flow of Sec. 3.1 by
non-equilibrium extrapolation) through the C ABI, against the FP64 oracle on
the same seeded inputs.

Tolerances: FP64 one step max |df| <= 1e-14 max |f| on every node (fluid
rows and velocity rows); FP64 long runs rel-L2(u) <= 1e-12 sqrt(steps/1000)
(rounding differences random-walk); FP32-shifted storage reported and bounded
by its storage rounding.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2409_02964_amd import workloads as W  # noqa: E402

RATES = dict(s_c=1.1, s_e=1.3, s_eps=1.2, s_q=1.4, s_nu=0.9)


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rates_for(nu):
    return dict(s_c=1.0, s_e=1.0 / (nu + 0.5), s_eps=1.2, s_q=1.4, s_nu=1.0 / (3 * nu + 0.5))


# (nx, ny, faces (u_lo, u_hi), eq2, drag, force, dynamic phi, tiling)
CASES = [
    (45, 23, (None, 3e-3), False, False, False, False, None),
    (45, 23, (-2e-3, None), True, True, False, False, (64, 5)),
    (37, 3, (1e-3, -2e-3), False, True, True, False, (64, 1)),      # one fluid row
    (130, 17, (2e-3, 4e-3), False, False, True, True, (128, 4)),
    (253, 12, (None, 1e-3), True, False, False, True, (256, 2)),
]


@pytest.mark.parametrize("nx,ny,rows,eq2,drag,force,dyn,tiling", CASES)
def test_one_step_velocity_rows_fp64(oracle, nx, ny, rows, eq2, drag, force, dyn, tiling):
    torch = _torch()
    from paper_2409_02964_amd.vanse import Lattice
    _say(f"velocity rows {nx}x{ny} rows={rows} eq2={eq2} drag={drag} force={force} dyn={dyn}")
    phi = 0.45 + 0.5 * W.smoothed_noise(nx, ny, 2.0, seed=nx + ny) ** 2
    phin = phi * (1.0 + 2e-3 * W.smoothed_noise(nx, ny, 3.0, seed=3)) if dyn else None
    beta = (2e-3 + 1e-2 * (1 - phi)) if drag else None
    fxy = (1e-5 * W.smoothed_noise(nx, ny, 2.0, seed=8),
           -1e-5 * W.smoothed_noise(nx, ny, 2.0, seed=9)) if force else None
    f0 = W.random_populations(nx, ny, seed=17 + nx)
    ora = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=RATES, g=(2e-5, -1e-5), bc_y="wall",
                        eq2=eq2, drag=None if beta is None else (beta, (1e-4, 0.0)),
                        force=fxy, velocity_rows=rows)
    ora.set_populations(f0)
    ora.step(1, phi_next=phin)
    lat = Lattice(nx, ny, precision="f64", bc_y="wall", drag=drag, force_field=force,
                  dynamic_phi=dyn)
    lat.set_params(0.5, RATES).set_body_force(2e-5, -1e-5).set_void_fraction(phi)
    if drag:
        lat.set_drag(beta, (1e-4, 0.0))
    if force:
        lat.set_force_field(*fxy)
    if tiling:
        lat.set_tiling(*tiling)
    lat.set_scheme("A", 2 if eq2 else 3).set_velocity_rows(*rows)
    lat.set_populations(torch.from_numpy(f0), rho0=1.0)
    if dyn:
        lat.set_void_fraction_next(phin)
    lat.step(1)
    fg = lat.read_populations().cpu().numpy()
    scale = np.max(np.abs(ora.f))
    err = np.max(np.abs(fg - ora.f)) / scale
    m = {k: v.cpu().numpy() for k, v in lat.read_moments().items()}
    ref = ora.macroscopic()
    em = max(np.max(np.abs(m["rho"] - ref["rho"])), np.max(np.abs(m["ux"] - ref["ux"])),
             np.max(np.abs(m["uy"] - ref["uy"])))
    _say(f"  populations max rel err {err:.3e}, moments max abs err {em:.3e}")
    assert err <= 1e-14
    assert em <= 1e-14
    for k, u in zip((0, ny - 1), rows):   # the rows report the wall velocity
        if u is not None:
            assert np.all(m["ux"][k] == u) and np.all(m["uy"][k] == 0.0)


@pytest.mark.parametrize("prec,bound", [("f64", 1e-12), ("f32s", 1e-4)])
def test_porous_couette_velocity_row(oracle, prec, bound):
    """Eq. (22) II as in Sec. 3.1: Brinkman drag (Da = 0.01), lower wall at
    rest (half-way), upper wall a velocity row at U; against the oracle over
    six viscous times and, coarsely, against the closed form."""
    _torch()
    from paper_2409_02964_amd.vanse import Lattice
    ny, nx, nu, phi0, U = 32, 8, 0.1, 0.5, 1e-3
    H = ny - 0.5
    k0 = 0.01 * H * H
    beta = np.full((ny, nx), phi0 * nu / k0)
    rates = _rates_for(nu)
    phi = np.full((ny, nx), phi0)
    ora = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=rates, bc_y="wall", drag=(beta, (0, 0)),
                        velocity_rows=(None, U)).init_equilibrium()
    lat = Lattice(nx, ny, precision=prec, bc_y="wall", drag=True)
    lat.set_params(0.5, rates).set_void_fraction(phi).set_drag(beta)
    lat.set_velocity_rows(None, U).init_equilibrium(1.0)
    steps = int(6 * H * H / nu)
    ora.step(steps)
    lat.step(steps)
    m = {k: v.cpu().numpy() for k, v in lat.read_moments().items()}
    ref = ora.macroscopic()
    e = math.sqrt(np.sum((m["ux"] - ref["ux"]) ** 2 + (m["uy"] - ref["uy"]) ** 2)
                  / np.sum(ref["ux"] ** 2 + ref["uy"] ** 2))
    y = np.arange(ny) + 0.5
    a = math.sqrt(phi0 / k0)
    exact = U * np.sinh(a * y) / math.sinh(a * H)
    e_exact = np.max(np.abs(m["ux"][:, 0] - exact)) / U
    _say(f"porous Couette (velocity row) {prec}: rel-L2(u) vs oracle {e:.3e}, "
         f"vs Eq. 22 {e_exact:.3e}")
    if prec == "f64":
        bound *= math.sqrt(steps / 1000.0)
    assert e <= bound
    assert e_exact < 1e-2


def test_couette_velocity_row_linear_f64(oracle):
    """Plain Couette flow between a half-way wall at rest and a velocity row
    at U, phi != kappa: the GPU's steady profile is the exact linear one."""
    _torch()
    from paper_2409_02964_amd.vanse import Lattice
    ny, nx, nu, U = 12, 64, 0.1, 1e-3
    lat = Lattice(nx, ny, precision="f64", bc_y="wall")
    lat.set_params(0.5, _rates_for(nu)).set_void_fraction(np.full((ny, nx), 0.8))
    lat.set_velocity_rows(None, U).init_equilibrium(1.0)
    lat.step(int(8 * (ny - 0.5) ** 2 / nu))
    u = lat.read_moments()["ux"].cpu().numpy()
    exact = U * (np.arange(ny) + 0.5) / (ny - 0.5)
    err = np.max(np.abs(u - exact[:, None])) / U
    _say(f"Couette (velocity row) linear profile: max rel err {err:.3e}")
    assert err < 1e-7


def test_velocity_rows_observables_skip_the_rows(oracle):
    """Mass and |u|^2 are sums over the fluid rows only."""
    torch = _torch()
    from paper_2409_02964_amd.vanse import Lattice
    nx, ny = 40, 10
    phi = 0.6 + 0.3 * W.smoothed_noise(nx, ny, 2.0, seed=4) ** 2
    f0 = W.random_populations(nx, ny, seed=5)
    ora = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=RATES, g=(1e-5, 0), bc_y="wall",
                        velocity_rows=(1e-3, -1e-3))
    ora.set_populations(f0)
    ora.step(3)
    lat = Lattice(nx, ny, precision="f64", bc_y="wall")
    lat.set_params(0.5, RATES).set_body_force(1e-5, 0).set_void_fraction(phi)
    lat.set_velocity_rows(1e-3, -1e-3).set_populations(torch.from_numpy(f0), rho0=1.0)
    lat.step(3)
    obs = lat.observe()
    ref = ora.macroscopic()
    fl = ora.fluid()
    assert abs(obs["mass"] - ora.mass()) <= 1e-13 * ora.mass()
    u2 = float(np.sum(ref["ux"][fl] ** 2 + ref["uy"][fl] ** 2))
    assert abs(obs["u2"] - u2) <= 1e-12 * u2


def test_velocity_rows_errors():
    _torch()
    from paper_2409_02964_amd.vanse import Batch, Lattice, VanseError
    phi = np.full((8, 16), 0.8)

    def lat(**kw):
        L = Lattice(16, 8, precision="f64", **kw)
        L.set_params(0.5, RATES).set_void_fraction(phi)
        return L

    with pytest.raises(VanseError):             # no walls
        lat().set_velocity_rows(None, 1e-3)
    with pytest.raises(VanseError):             # walls in x
        lat(bc_y="wall", bc_x="wall").set_velocity_rows(None, 1e-3)
    with pytest.raises(VanseError):             # solid nodes
        lat(bc_y="wall", mask=True).set_velocity_rows(None, 1e-3)
    a = lat(bc_y="wall").set_wall_velocity(0.0, 1e-3)
    with pytest.raises(VanseError):             # the half-way wall already moves
        a.set_velocity_rows(None, 1e-3)
    a.set_velocity_rows(1e-3, None)             # the other face is free
    with pytest.raises(VanseError):
        a.set_wall_velocity(2e-3, 1e-3)
    a.init_equilibrium(1.0)
    with pytest.raises(VanseError):             # fixed once populations exist
        a.set_velocity_rows(None, None)
    with pytest.raises(VanseError):             # batches do not take them
        Batch([a])
