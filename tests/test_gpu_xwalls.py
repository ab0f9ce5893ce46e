"""GPU parity of walls in x (half-way bounce-back at x = -1/2 and x = nx - 1/2)
through the C ABI, against the FP64 oracle on the same seeded inputs.

Walls in x run the solid-node kernel instances: the face columns pull across
the face from their own opposite slots, and the halo lanes beyond a face stand
for the mirror column (scalars copied, velocity-like fields negated).  The
shapes put the faces in the first and in a ragged last strip, and in one
strip together.  Tolerances as for the other variants: FP64 one step
max|df| <= 1e-14 max|f|; FP64 many steps rel-L2(u) <= 1e-12.
"""
import math
import sys

import numpy as np
import pytest

from paper_2409_02964_amd import workloads as W

pytestmark = pytest.mark.gpu

C1_RATES = dict(s_c=1.2, s_e=1.2, s_eps=1.2, s_q=1.2, s_nu=0.8)


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2_u(m, ref, fluid=None):
    sel = np.ones_like(ref["ux"], bool) if fluid is None else fluid
    num = np.sum((m["ux"][sel] - ref["ux"][sel]) ** 2 + (m["uy"][sel] - ref["uy"][sel]) ** 2)
    den = np.sum(ref["ux"][sel] ** 2 + ref["uy"][sel] ** 2)
    return math.sqrt(num / den)


def to_np(d):
    return {k: v.cpu().numpy() for k, v in d.items()}


SWAP = [0, 2, 1, 4, 3, 5, 8, 7, 6]  # direction of (e_y, e_x) for direction i of (e_x, e_y)


def xlattice(nx, ny, phi, precision="f64", bc_y="periodic", mask=None, force=None, drag=None,
             dynamic=False, g=(0.0, 0.0), tiling=None):
    from paper_2409_02964_amd.vanse import Lattice
    lat = Lattice(nx, ny, precision=precision, bc_x="wall", bc_y=bc_y, mask=mask is not None,
                  force_field=force is not None, drag=drag is not None, dynamic_phi=dynamic)
    lat.set_params(0.5, C1_RATES).set_body_force(g[0], g[1], True)
    if mask is not None:
        lat.set_mask(mask)
    lat.set_void_fraction(phi)
    if force is not None:
        lat.set_force_field(force[0], force[1])
    if drag is not None:
        lat.set_drag(drag[0], drag[1])
    if tiling:
        lat.set_tiling(*tiling)
    return lat


SHAPES = [  # nx, ny, bc_y, tiling, mask, coupled (force field and drag)
    (61, 37, "periodic", None, False, False),
    (130, 20, "wall", (64, 5), False, False),     # three strips, the last 10 wide
    (66, 12, "periodic", (64, 4), True, False),   # the last strip 6 wide
    (200, 16, "wall", (128, 3), True, True),
    (8, 9, "wall", None, False, True),            # both faces in one strip
]


@pytest.mark.parametrize("nx,ny,bc,tiling,with_mask,coupled", SHAPES)
def test_one_step_x_walls_fp64(oracle, nx, ny, bc, tiling, with_mask, coupled):
    torch = _torch()
    _say(f"one-step x-walls fp64 {nx}x{ny} bc_y={bc} tiling={tiling} mask={with_mask} coupled={coupled}")
    phi = 0.55 + 0.4 * W.smoothed_noise(nx, ny, 2.0, seed=nx + 5 * ny) ** 2
    mask = W.solid_mask(nx, ny, seed=nx) if with_mask else None
    fluid = np.ones((ny, nx), bool) if mask is None else mask == 0
    f0 = W.random_populations(nx, ny, seed=3 + nx)
    g = (2e-5, -1e-5)
    force = drag = None
    if coupled:
        force = (2e-6 * W.smoothed_noise(nx, ny, 3.0, seed=41), -1e-6 * W.smoothed_noise(nx, ny, 3.0, seed=42))
        drag = (1e-3 + 2e-2 * (1 - phi), (3e-4, -1e-4))
    ora = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=C1_RATES, g=g, bc_x="wall", bc_y=bc,
                        mask=mask, force=force, drag=drag)
    ora.set_populations(f0)
    ora.step(1)
    lat = xlattice(nx, ny, phi, "f64", bc, mask=mask, force=force, drag=drag, g=g, tiling=tiling)
    lat.set_populations(torch.from_numpy(f0))
    back = lat.read_populations().cpu().numpy()
    assert np.max(np.abs(back[:, fluid] - f0[:, fluid])) <= 1e-15 * np.max(np.abs(f0))
    lat.step(1)
    fg = lat.read_populations().cpu().numpy()
    err = np.max(np.abs(fg[:, fluid] - ora.f[:, fluid])) / np.max(np.abs(ora.f))
    _say(f"   max rel err {err:.3e}")
    assert err <= 1e-14
    mg, mo = to_np(lat.read_moments()), ora.macroscopic()
    assert rel_l2_u(mg, mo, fluid) <= 1e-13  # the read-out's Eq. 10 across x faces


def test_box_many_steps_fp64(oracle):
    """A closed box (walls on all four sides) with solid grains, driven by a
    body force: 400 steps against the oracle, and mass conserved."""
    torch = _torch()
    nx, ny, steps = 64, 48, 400
    phi = 0.55 + 0.4 * W.smoothed_noise(nx, ny, 4.0, seed=11) ** 2
    mask = W.solid_mask(nx, ny, seed=13)
    fluid = mask == 0
    g = (2e-6, 1e-6)
    ora = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=C1_RATES, g=g, bc_x="wall", bc_y="wall",
                        mask=mask).init_equilibrium()
    ora.step(steps)
    ref = ora.macroscopic()
    lat = xlattice(nx, ny, phi, "f64", "wall", mask=mask, g=g)
    lat.init_equilibrium(1.0)
    obs0 = lat.observe()
    lat.step(steps)
    # the flow relaxes towards rest (|u| ~ 1e-7), so the populations are compared
    fg = lat.read_populations().cpu().numpy()
    err = np.max(np.abs(fg[:, fluid] - ora.f[:, fluid])) / np.max(np.abs(ora.f))
    m = to_np(lat.read_moments())
    du = np.max(np.abs(m["ux"] - ref["ux"])[fluid])
    obs = lat.observe()
    _say(f"box fp64: max rel err {err:.3e}, max|du| {du:.2e} (max|u| {np.max(np.abs(ref['ux'])):.2e}), "
         f"mass drift {abs(obs['mass'] - obs0['mass']) / obs0['mass']:.2e}")
    assert err <= 1e-13
    assert du <= 1e-15
    assert abs(obs["mass"] - obs0["mass"]) <= 1e-13 * obs0["mass"]


def test_box_at_rest_under_force_along_walls_fp64(oracle):
    """Hydrostatic equilibrium along the walls (the oracle's pin of the
    Eq. 10 stand-in beyond a wall, tests/test_oracle_wall_pins.py): a closed
    box under phi G along x, phi varying along x, stays at rest on the GPU and
    its rho depends on x alone; the populations match the oracle's."""
    torch = _torch()
    from paper_2409_02964_amd.vanse import Lattice
    nx, ny, steps, G = 24, 10, 6000, 1e-5
    rates = dict(s_c=1.0, s_e=1.2, s_eps=1.2, s_q=1.2, s_nu=1.0)
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    phi = 0.6 + 0.3 * np.sin(np.pi * (x + 0.5) / nx) ** 2
    _say(f"box at rest fp64 {nx}x{ny}, {steps} steps")
    ora = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=rates, g=(G, 0.0), bc_x="wall",
                        bc_y="wall").init_equilibrium()
    ora.step(steps)
    lat = Lattice(nx, ny, precision="f64", bc_x="wall", bc_y="wall")
    lat.set_params(0.5, rates).set_body_force(G, 0.0, True).set_void_fraction(phi)
    lat.init_equilibrium(1.0)
    lat.step(steps)
    m = to_np(lat.read_moments())
    fg = lat.read_populations().cpu().numpy()
    err = np.max(np.abs(fg - ora.f)) / np.max(np.abs(ora.f))
    urel = max(np.max(np.abs(m["ux"])), np.max(np.abs(m["uy"]))) / G
    spread = np.max(np.abs(m["rho"] - m["rho"][ny // 2][None, :])) / (G * nx)
    _say(f"box at rest fp64: max rel err {err:.3e}, max|u|/G {urel:.2e}, rho spread across y {spread:.2e}")
    assert err <= 1e-13
    assert urel < 1e-7
    assert spread < 1e-9


def test_lid_driven_cavity_fp64(oracle):
    """Walls on all four sides, the upper one moving at 0.01: 400 steps
    against the oracle (the moving-wall corrections meet the x-walls at the
    upper corners)."""
    torch = _torch()
    nx, ny, steps = 64, 64, 400
    phi = 0.7 + 0.25 * W.smoothed_noise(nx, ny, 4.0, seed=15) ** 2
    ora = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=C1_RATES, bc_x="wall", bc_y="wall",
                        wall_velocity=(0.0, 1e-2), rho_w=1.0).init_equilibrium()
    ora.step(steps)
    ref = ora.macroscopic()
    lat = xlattice(nx, ny, phi, "f64", "wall")
    lat.set_wall_velocity(0.0, 1e-2)
    lat.init_equilibrium(1.0).step(steps)
    e = rel_l2_u(to_np(lat.read_moments()), ref)
    _say(f"lid-driven cavity fp64: rel-L2(u) {e:.3e}, max|u| {np.max(np.abs(ref['ux'])):.2e}")
    assert e <= 1e-12


@pytest.mark.parametrize("model,order,uw", [("B", 3, (0.0, 0.0)), ("A", 2, (0.0, 0.0)),
                                            ("A", 3, (3e-3, -2e-3))])
def test_one_step_x_walls_scheme_variants_fp64(oracle, model, order, uw):
    """Model B, the Appendix B equilibrium and moving y-walls next to walls in
    x (the corners take both mirror images)."""
    torch = _torch()
    nx, ny = 45, 23
    _say(f"one-step x-walls scheme {model}/{order} uw={uw}")
    phi = 0.55 + 0.4 * W.smoothed_noise(nx, ny, 2.5, seed=51) ** 2
    f0 = W.random_populations(nx, ny, seed=52)
    ora = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=C1_RATES, g=(1e-5, 2e-6), bc_x="wall",
                        bc_y="wall", model_b=model == "B", eq2=order == 2, wall_velocity=uw,
                        rho_w=1.0)
    ora.set_populations(f0)
    ora.step(1)
    lat = xlattice(nx, ny, phi, "f64", "wall", g=(1e-5, 2e-6))
    lat.set_scheme(model, order)
    if uw != (0.0, 0.0):
        lat.set_wall_velocity(*uw)
    lat.set_populations(torch.from_numpy(f0), rho0=1.0).step(1)
    fg = lat.read_populations().cpu().numpy()
    err = np.max(np.abs(fg - ora.f)) / np.max(np.abs(ora.f))
    _say(f"   max rel err {err:.3e}")
    assert err <= 1e-14


def test_one_step_x_walls_dynamic_phi_fp64(oracle):
    torch = _torch()
    nx, ny = 50, 30
    phi = 0.55 + 0.4 * W.smoothed_noise(nx, ny, 3.0, seed=61) ** 2
    phin = np.clip(phi + 0.02 * W.smoothed_noise(nx, ny, 3.0, seed=62), 0.3, 1.0)
    f0 = W.random_populations(nx, ny, seed=63)
    ora = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=C1_RATES, g=(1e-5, 0), bc_x="wall")
    ora.set_populations(f0)
    ora.step(1, phi_next=phin)
    lat = xlattice(nx, ny, phi, "f64", dynamic=True, g=(1e-5, 0))
    lat.set_populations(torch.from_numpy(f0))
    lat.set_void_fraction_next(phin)
    lat.step(1)
    err = np.max(np.abs(lat.read_populations().cpu().numpy() - ora.f)) / np.max(np.abs(ora.f))
    _say(f"one-step x-walls dynamic phi: max rel err {err:.3e}")
    assert err <= 1e-14


def test_x_walls_are_transposed_y_walls_gpu():
    """The x-wall kernel path on transposed inputs reproduces the transpose of
    the plain y-wall path (another instance, another code path)."""
    torch = _torch()
    from paper_2409_02964_amd.vanse import Lattice
    nx, ny, steps = 96, 40, 100
    phi = 0.55 + 0.4 * W.smoothed_noise(nx, ny, 3.0, seed=71) ** 2
    f0 = W.random_populations(nx, ny, seed=72)
    a = Lattice(nx, ny, precision="f64", bc_y="wall")
    a.set_params(0.5, C1_RATES).set_body_force(2e-6, -1e-6, True).set_void_fraction(phi)
    a.set_populations(torch.from_numpy(f0)).step(steps)
    b = xlattice(ny, nx, phi.T.copy(), "f64", g=(-1e-6, 2e-6))
    b.set_populations(torch.from_numpy(np.stack([f0[SWAP[i]].T for i in range(9)]))).step(steps)
    fa = a.read_populations().cpu().numpy()
    fb = b.read_populations().cpu().numpy()
    err = np.max(np.abs(np.stack([fa[SWAP[i]].T for i in range(9)]) - fb)) / np.max(np.abs(fa))
    _say(f"x-walls vs transposed y-walls, {steps} steps: {err:.3e}")
    assert err <= 1e-13


def test_x_walls_shifted_fp32(oracle):
    torch = _torch()
    nx, ny, steps = 96, 40, 300
    phi = 0.55 + 0.4 * W.smoothed_noise(nx, ny, 4.0, seed=81) ** 2
    ora = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=C1_RATES, g=(2e-6, 1e-6), bc_x="wall",
                        bc_y="wall").init_equilibrium()
    ora.step(steps)
    lat = xlattice(nx, ny, phi, "f32s", "wall", g=(2e-6, 1e-6))
    lat.init_equilibrium(1.0).step(steps)
    e = rel_l2_u(to_np(lat.read_moments()), ora.macroscopic())
    _say(f"x-walls f32s {steps} steps: rel-L2(u) {e:.3e}")
    assert e <= 1e-4


def test_x_walls_two_steps_per_launch_fall_back(oracle):
    """Two steps per launch are not built for walls in x: the lattice steps
    one at a time, with the same results."""
    torch = _torch()
    nx, ny = 70, 30
    phi = 0.6 + 0.3 * W.smoothed_noise(nx, ny, 3.0, seed=91) ** 2
    f0 = W.random_populations(nx, ny, seed=92)
    ora = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=C1_RATES, g=(1e-5, 0), bc_x="wall", bc_y="wall")
    ora.set_populations(f0)
    ora.step(5)
    lat = xlattice(nx, ny, phi, "f64", "wall", g=(1e-5, 0))
    lat.set_steps_per_pass(2)
    lat.set_populations(torch.from_numpy(f0)).step(5)
    err = np.max(np.abs(lat.read_populations().cpu().numpy() - ora.f)) / np.max(np.abs(ora.f))
    assert err <= 1e-14


def test_x_walls_batch_bitwise():
    """Members with walls in x batched: bitwise the results of stepping each
    alone; members differing in bc_x are refused."""
    _torch()
    from paper_2409_02964_amd.vanse import Batch, Lattice, VanseError
    sizes = [(64, 48), (37, 53), (130, 20)]

    def member(k, nx, ny, bc_x="wall", mask=True):
        lat = Lattice(nx, ny, precision="f32s", bc_x=bc_x, bc_y="wall", mask=mask)
        phi = 0.6 + 0.3 * np.sin(2 * np.pi * np.arange(nx)[None, :] / nx) * np.cos(2 * np.pi * np.arange(ny)[:, None] / ny)
        lat.set_params(0.5, C1_RATES).set_body_force(1e-6 * (k + 1), 2e-7)
        if mask:
            lat.set_mask(W.solid_mask(nx, ny, seed=k))
        lat.set_void_fraction(phi)
        return lat.init_equilibrium(1.0, 1e-3, 0.0)

    ref = [member(k, nx, ny) for k, (nx, ny) in enumerate(sizes)]
    for lat in ref:
        lat.step(11)
    mem = [member(k, nx, ny) for k, (nx, ny) in enumerate(sizes)]
    Batch(mem, threads=64, rows=7, graph_steps=0).step(11)
    for a, r in zip(mem, ref):
        assert np.array_equal(a.read_populations().cpu().numpy(), r.read_populations().cpu().numpy())
    with pytest.raises(VanseError):
        Batch([member(0, 40, 30), member(1, 40, 30, bc_x="periodic")])


@pytest.mark.parametrize("mask", [False, True])
def test_x_walls_batch_force_drag_bitwise(mask):
    """Walls in x with a force field and a drag take the moving-phi instance
    (with or without solid nodes); batched, they are bitwise the results of
    stepping each member alone."""
    _torch()
    from paper_2409_02964_amd.vanse import Batch, Lattice
    sizes = [(64, 48), (37, 53), (130, 20)]

    def member(k, nx, ny):
        lat = Lattice(nx, ny, precision="f32s", bc_x="wall", bc_y="wall", mask=mask,
                      force_field=True, drag=True)
        phi = 0.55 + 0.4 * W.smoothed_noise(nx, ny, 3.0, seed=k + 7) ** 2
        lat.set_params(0.5, C1_RATES).set_body_force(1e-6 * (k + 1), 2e-7)
        if mask:
            lat.set_mask(W.solid_mask(nx, ny, seed=k))
        lat.set_void_fraction(phi)
        lat.set_force_field(1e-6 * W.smoothed_noise(nx, ny, 3.0, seed=k + 20),
                            -1e-6 * W.smoothed_noise(nx, ny, 3.0, seed=k + 30))
        lat.set_drag(1e-3 + 1e-2 * (1 - phi), (1e-4, 0.0))
        return lat.init_equilibrium(1.0, 1e-3, 0.0)

    ref = [member(k, nx, ny) for k, (nx, ny) in enumerate(sizes)]
    for lat in ref:
        lat.step(9)
    mem = [member(k, nx, ny) for k, (nx, ny) in enumerate(sizes)]
    Batch(mem, threads=64, rows=6, graph_steps=0).step(9)
    for a, r in zip(mem, ref):
        assert np.array_equal(a.read_populations().cpu().numpy(), r.read_populations().cpu().numpy())


@pytest.mark.parametrize("prec,bound", [("f16s", 2e-2), ("f32", 2e-3)])
def test_x_walls_reduced_storage(oracle, prec, bound):
    """A closed box in FP16-shifted and plain FP32 storage against the FP64
    oracle: the error is the storage rounding's, reported."""
    _torch()
    nx, ny, steps = 96, 40, 300
    phi = 0.55 + 0.4 * W.smoothed_noise(nx, ny, 4.0, seed=81) ** 2
    ora = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=C1_RATES, g=(2e-6, 1e-6), bc_x="wall",
                        bc_y="wall").init_equilibrium()
    ora.step(steps)
    lat = xlattice(nx, ny, phi, prec, "wall", g=(2e-6, 1e-6))
    lat.init_equilibrium(1.0).step(steps)
    e = rel_l2_u(to_np(lat.read_moments()), ora.macroscopic())
    _say(f"x-walls {prec} {steps} steps: rel-L2(u) {e:.3e}")
    assert e <= bound
