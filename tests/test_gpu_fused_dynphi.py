"""Two time steps per launch with a moving void fraction (the d_t phi term of
Eq. 20; the moving particles of Eq. 23): vanse_set_void_fraction_next2 hands
over phi(t+1), phi(t+2) and, when they change, the second step's drag
coefficient and force field.

The oracle takes the same inputs one step at a time (phi_next, and its drag
and force arrays rewritten between the steps).  Tolerances: FP64 max |df| <=
1e-14 max |f| after one launch and 1e-13 after several; rel-L2(u) <= 1e-12
over long runs; FP32-shifted and FP16-shifted against one step per launch as
in the other two-step tests, and against the oracle at the bounds of the
single step.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2409_02964_amd import workloads as W  # noqa: E402

RATES = dict(s_c=1.2, s_e=1.2, s_eps=1.2, s_q=1.2, s_nu=0.8)
FUSED_RTOL = 1e-5


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def lattice(nx, ny, phi, precision="f64", bc="periodic", fused=True, rows=0, g=(1e-5, 0.0),
            force=None, drag=None, scale_by_phi=True, kappa=0.5, rates=RATES):
    from paper_2409_02964_amd.vanse import Lattice
    lat = Lattice(nx, ny, precision=precision, bc_y=bc, dynamic_phi=True, force_field=force is not None,
                  drag=drag is not None)
    lat.set_params(kappa, rates).set_body_force(g[0], g[1], scale_by_phi).set_void_fraction(phi)
    if force is not None:
        lat.set_force_field(*force)
    if drag is not None:
        lat.set_drag(*drag)
    if fused:
        lat.set_steps_per_pass(2, rows)
    return lat


def rel_l2_u(m, ref):
    num = np.sum((m["ux"] - ref["ux"]) ** 2 + (m["uy"] - ref["uy"]) ** 2)
    return math.sqrt(num / np.sum(ref["ux"] ** 2 + ref["uy"] ** 2))


def to_np(d):
    return {k: v.cpu().numpy() for k, v in d.items()}


def moving_fields(nx, ny, t, with_beta, with_force):
    """Seeded smooth inputs of step t: phi(t) in [0.35, 0.95] drifting in x,
    beta(t) = 1e-3 + 2e-2 (1 - phi(t)), a force field changing with t."""
    base = W.smoothed_noise(nx, ny, 3.0, seed=21)
    wave = np.sin(2 * np.pi * (np.arange(nx)[None, :] - 0.7 * t) / nx) * np.ones((ny, 1))
    phi = np.clip(0.65 + 0.15 * base + 0.12 * wave, 0.35, 0.95)
    beta = 1e-3 + 2e-2 * (1 - phi) if with_beta else None
    force = None
    if with_force:
        ph = 0.1 * t
        force = (2e-6 * np.cos(ph) * W.smoothed_noise(nx, ny, 3.0, seed=23),
                 -1e-6 * np.sin(ph + 0.3) * W.smoothed_noise(nx, ny, 3.0, seed=24))
    return phi, beta, force


@pytest.mark.parametrize("nx,ny,bc,rows,drag,force", [
    (48, 40, "periodic", 0, False, False), (61, 37, "wall", 0, False, False),
    (61, 37, "wall", 5, True, False), (130, 44, "periodic", 3, True, True),
    (64, 32, "wall", 0, False, True), (7, 6, "periodic", 0, True, False)])
def test_fused_dynphi_fp64_vs_oracle(oracle, nx, ny, bc, rows, drag, force):
    torch = _torch()
    _say(f"fused moving phi fp64 {nx}x{ny} {bc} rows={rows} drag={drag} force={force}")
    phi0, beta0, f0c = moving_fields(nx, ny, 0, drag, force)
    us = (3e-4, -1e-4)
    ora = oracle.Oracle(nx, ny, phi0, kappa=0.5, rates=RATES, g=(1e-5, 0), bc_y=bc,
                        force=f0c, drag=None if beta0 is None else (beta0, us))
    pops = W.random_populations(nx, ny, seed=31 + nx)
    ora.set_populations(pops)
    lat = lattice(nx, ny, phi0, "f64", bc, rows=rows, force=f0c,
                  drag=None if beta0 is None else (beta0, us))
    assert lat.fused_tiling()["active"]
    lat.set_populations(torch.from_numpy(pops))
    for launch in range(3):
        t = 2 * launch
        p1, b1, f1 = moving_fields(nx, ny, t + 1, drag, force)
        p2, _, _ = moving_fields(nx, ny, t + 2, drag, force)
        ora.step(1, phi_next=p1)
        if drag:
            ora.beta[...] = b1
        if force:
            ora.fx[...] = f1[0]
            ora.fy[...] = f1[1]
        ora.step(1, phi_next=p2)
        lat.set_void_fraction_next2(p1, p2, beta_next=b1, force_next=f1)
        lat.step(2)
        fg = lat.read_populations().cpu().numpy()
        err = np.max(np.abs(fg - ora.f)) / np.max(np.abs(ora.f))
        _say(f"   t={lat.t}: max rel err {err:.3e}")
        assert err <= (1e-14 if launch == 0 else 1e-13)
    mg, mo = to_np(lat.read_moments()), ora.macroscopic()
    assert np.max(np.abs(mg["rho"] - mo["rho"])) <= 1e-13  # phi(t+2) is current


def _mms3_fused(oracle, n, precision, steps, a=0.5, b=0.25, nu=0.1, kappa=0.3, us=0.08):
    """MMS case III (Eq. 29: moving phi and velocity, Appendix C force) with
    two steps per launch against the oracle stepped one step at a time."""
    torch = _torch()
    s_nu = 1.0 / (3 * nu + 0.5)
    rates = dict(s_c=1.0, s_e=1.0 / (nu + 0.5), s_eps=1.2, s_q=1.2, s_nu=s_nu)
    m0 = W.mms_case("III", n, a, b, us, nu, 0)
    ora = oracle.Oracle(n, n, m0["phi"], kappa=kappa, rates=rates, scale_by_phi=False,
                        force=(m0["fx"], m0["fy"]))
    ora.init_fields(np.ones((n, n)), m0["ux"], m0["uy"])
    lat = lattice(n, n, m0["phi"], precision, force=(m0["fx"], m0["fy"]), g=(0.0, 0.0),
                  scale_by_phi=False, kappa=kappa, rates=rates)
    assert lat.fused_tiling()["active"]
    lat.set_populations(torch.from_numpy(ora.f.copy()))
    for t in range(0, steps, 2):
        m0 = W.mms_case("III", n, a, b, us, nu, t)
        m1 = W.mms_case("III", n, a, b, us, nu, t + 1)
        m2 = W.mms_case("III", n, a, b, us, nu, t + 2)
        for mt, mn in ((m0, m1), (m1, m2)):
            ora.fx[...] = mt["fx"]
            ora.fy[...] = mt["fy"]
            ora.step(1, phi_next=mn["phi"])
        # the force field of step t, then that of step t + 1 with the hand-over
        lat.set_force_field(m0["fx"], m0["fy"])
        lat.set_void_fraction_next2(m1["phi"], m2["phi"], force_next=(m1["fx"], m1["fy"]))
        lat.step(2)
    return to_np(lat.read_moments()), ora.macroscopic()


def test_fused_mms_case_III_fp64(oracle):
    m, ref = _mms3_fused(oracle, 32, "f64", 200)
    e = rel_l2_u(m, ref)
    _say(f"MMS III fp64, two steps per launch, 200 steps: rel-L2(u) {e:.3e}")
    assert e <= 1e-12


@pytest.mark.parametrize("prec,bound", [("f32s", 1e-4), ("f16s", 2e-2)])
def test_fused_mms_case_III_shifted_storage(oracle, prec, bound):
    m, ref = _mms3_fused(oracle, 32, prec, 200)
    e = rel_l2_u(m, ref)
    _say(f"MMS III {prec}, two steps per launch, 200 steps: rel-L2(u) {e:.3e}")
    assert e <= bound


def test_fused_particle_flow_eq23_fp64(oracle):
    """Sec. 3.2, Eq. (23): a travelling void fraction phi(x, t) = 1 + a(sin(2 pi
    (x - u_s t)/L) - 1) with F^B = phi (G - phi (1 - phi)(u - u_s)): the
    body force scaled by phi and the drag beta = phi (1 - phi), both moving
    with phi.  Two steps per launch against the oracle over 400 steps; kappa
    at the smallest void fraction, 1 - 2a (Sec. 2.3: with kappa = 0.5 this
    field diverges in the oracle as well)."""
    _torch()
    L, H, a, us, G, steps = 100, 5, 0.45, 1e-3, 1e-6, 400
    kappa = 1 - 2 * a
    x = np.arange(L)[None, :] + 0.5

    def phi_at(t):
        return (1 + a * (np.sin(2 * np.pi * (x - us * t) / L) - 1)) * np.ones((H, 1))

    p0 = phi_at(0)
    ora = oracle.Oracle(L, H, p0, kappa=kappa, rates=RATES, g=(G, 0.0), drag=(p0 * (1 - p0), (us, 0.0)))
    ora.init_equilibrium()
    lat = lattice(L, H, p0, "f64", g=(G, 0.0), drag=(p0 * (1 - p0), (us, 0.0)), kappa=kappa)
    lat.init_equilibrium(1.0)
    for t in range(0, steps, 2):
        p1, p2 = phi_at(t + 1), phi_at(t + 2)
        ora.step(1, phi_next=p1)
        ora.beta[...] = p1 * (1 - p1)
        ora.step(1, phi_next=p2)
        ora.beta[...] = p2 * (1 - p2)
        lat.set_void_fraction_next2(p1, p2, beta_next=p1 * (1 - p1))
        lat.step(2)
        lat.set_drag(p2 * (1 - p2), (us, 0.0))
    m, ref = to_np(lat.read_moments()), ora.macroscopic()
    e = rel_l2_u(m, ref)
    _say(f"Eq. 23 particle flow, two steps per launch: rel-L2(u) vs oracle {e:.3e}")
    assert e <= 1e-12


@pytest.mark.parametrize("prec,bc,drag,force", [("f32s", "wall", True, False), ("f32s", "periodic", False, True),
                                                ("f16s", "wall", True, False), ("f64", "periodic", True, True)])
def test_fused_dynphi_matches_single_steps(prec, bc, drag, force):
    """The same hand-over stepped with one step per launch: to FP32 rounding
    (FP64 to FP64 rounding; FP16-shifted about one storage rounding)."""
    torch = _torch()
    nx, ny = 253, 70
    phi0, beta0, f0c = moving_fields(nx, ny, 0, drag, force)
    pops = W.random_populations(nx, ny, seed=37)
    dr = None if beta0 is None else (beta0, (2e-4, 0.0))
    a = lattice(nx, ny, phi0, prec, bc, fused=False, force=f0c, drag=dr)
    b = lattice(nx, ny, phi0, prec, bc, fused=True, force=f0c, drag=dr)
    assert b.fused_tiling()["active"] and not a.fused_tiling()["active"]
    a.set_populations(torch.from_numpy(pops))
    b.set_populations(torch.from_numpy(pops))
    for launch in range(4):
        t = 2 * launch
        p1, b1, f1 = moving_fields(nx, ny, t + 1, drag, force)
        p2, _, _ = moving_fields(nx, ny, t + 2, drag, force)
        for lat in (a, b):
            lat.set_void_fraction_next2(p1, p2, beta_next=b1, force_next=f1)
        a.step(1)  # one step at a time, as two callers of one step would
        a.step(1)
        b.step(2)
    fa, fb = a.read_populations().cpu().numpy(), b.read_populations().cpu().numpy()
    rel = float(np.abs(fa - fb).max() / np.abs(fa - pops).max())
    _say(f"moving phi {prec} {bc}: fused vs single relative difference {rel:.3e}")
    assert rel <= {"f32s": FUSED_RTOL, "f16s": 2e-3, "f64": 1e-12}[prec]


def test_dynphi_two_pending_steps_errors():
    _torch()
    from paper_2409_02964_amd.vanse import Lattice, VanseError
    n = 16
    phi = np.full((n, n), 0.7)
    lat = lattice(n, n, phi, "f64", drag=(np.full((n, n), 1e-3), (0.0, 0.0)))
    lat.init_equilibrium(1.0)
    lat.set_void_fraction_next2(phi * 0.99, phi * 0.98)
    with pytest.raises(VanseError):  # at most the two pending steps
        lat.step(3)
    with pytest.raises(VanseError):  # phi(t) cannot be replaced while steps are pending
        lat.set_void_fraction(phi)
    with pytest.raises(VanseError):  # nor more void fractions handed over
        lat.set_void_fraction_next(phi)
    lat.step(2)
    assert lat.t == 2
    with pytest.raises(VanseError):  # both force planes or neither (and this lattice has none)
        lat.set_void_fraction_next2(phi, phi, force_next=(phi, phi))
    plain = lattice(n, n, phi, "f64")
    plain.init_equilibrium(1.0)
    with pytest.raises(VanseError):  # no drag on this lattice
        plain.set_void_fraction_next2(phi, phi, beta_next=phi)
    static = Lattice(n, n, "f64")
    static.set_params(0.5, RATES).set_void_fraction(phi).init_equilibrium(1.0)
    with pytest.raises(VanseError):  # needs dynamic_phi
        static.set_void_fraction_next2(phi, phi)
