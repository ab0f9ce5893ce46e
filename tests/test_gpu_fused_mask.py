"""Two time steps per launch with solid nodes (half-way bounce-back on their
faces and the centre-value stand-ins of the Eq. (10) stencils, Sec. 2.3).

The two-step kernel leaves solid nodes out of its separable stencil sums and
restores their stand-ins with the flagged-neighbour sums Kx, Ky; the pull
bounces back through per-lane offsets (first step) and ring selects (second
step).  Checks, on the seeded masks of the one-step tests (discs, isolated
solid nodes, solid nodes on the edge rows and columns next to walls and
periodic seams):
  - FP64 against the oracle: max |df| <= 1e-14 max |f| on fluid nodes after
    one launch (the one-step bar: the two kernels differ by FP64 roundings of
    the stencil sums), rel-L2(u) <= 1e-12 after many steps;
  - FP32-shifted and FP16-shifted against one step per launch on fluid nodes
    (the tolerances of the plain two-step tests);
  - solid nodes hold the rest state bitwise;
  - a batch with two steps per launch gives bitwise what each member gives
    alone with two steps per launch.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2409_02964_amd import workloads as W  # noqa: E402

RATES = dict(s_c=1.2, s_e=1.2, s_eps=1.2, s_q=1.2, s_nu=0.8)
FUSED_RTOL = 1e-5      # FP32-shifted against one step per launch (test_gpu_fused)
FUSED_RTOL16 = 2e-3    # FP16-shifted: about one storage rounding of the change


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def lattice(nx, ny, phi, mask, precision="f64", bc="periodic", fused=True, rows=0, g=(2e-5, -1e-5),
            force=None, drag=None):
    from paper_2409_02964_amd.vanse import Lattice
    lat = Lattice(nx, ny, precision=precision, bc_y=bc, mask=True, force_field=force is not None,
                  drag=drag is not None)
    lat.set_params(0.5, RATES).set_body_force(*g).set_mask(mask).set_void_fraction(phi)
    if force is not None:
        lat.set_force_field(*force)
    if drag is not None:
        lat.set_drag(*drag)
    if fused:
        lat.set_steps_per_pass(2, rows)
    return lat


def rel_l2_u(m, ref, fluid):
    num = np.sum((m["ux"][fluid] - ref["ux"][fluid]) ** 2 + (m["uy"][fluid] - ref["uy"][fluid]) ** 2)
    return math.sqrt(num / np.sum(ref["ux"][fluid] ** 2 + ref["uy"][fluid] ** 2))


def fluid_rel_diff(fa, fb, f0, fluid):
    """max |fa - fb| / max |fa - f0| over the fluid nodes"""
    return float(np.abs(fa[:, fluid] - fb[:, fluid]).max() / np.abs(fa[:, fluid] - f0[:, fluid]).max())


def field(nx, ny, seed):
    return 0.55 + 0.4 * W.smoothed_noise(nx, ny, 2.0, seed=seed) ** 2


# FP64 halves of 128 lanes output 118 columns: 300 columns take three strips
SHAPES = [
    (64, 48, "periodic", 0),
    (61, 37, "wall", 0),
    (253, 9, "periodic", 4),    # solid nodes on both sides of strip seams
    (125, 30, "wall", 7),
    (60, 5, "wall", 1),         # one row per workgroup
    (300, 70, "wall", 0),
    (130, 67, "periodic", 3),
    (7, 6, "periodic", 0),      # everything wraps
]


@pytest.mark.parametrize("nx,ny,bc,rows", SHAPES)
def test_fused_mask_fp64_vs_oracle(oracle, nx, ny, bc, rows):
    torch = _torch()
    _say(f"fused mask fp64 vs oracle {nx}x{ny} {bc} rows={rows}")
    phi = field(nx, ny, nx + 7 * ny)
    mask = W.solid_mask(nx, ny, seed=nx * ny + 1)
    fluid = mask == 0
    f0 = W.random_populations(nx, ny, seed=19 + nx)
    g = (2e-5, -1e-5)
    ora = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=RATES, g=g, bc_y=bc, mask=mask)
    ora.set_populations(f0)
    lat = lattice(nx, ny, phi, mask, "f64", bc, rows=rows, g=g)
    assert lat.fused_tiling()["active"]
    lat.set_populations(torch.from_numpy(f0))
    for n, bound in ((2, 1e-14), (5, 1e-13)):  # one launch; two launches and a single step
        ora.step(n)
        lat.step(n)
        fg = lat.read_populations().cpu().numpy()
        err = np.max(np.abs(fg[:, fluid] - ora.f[:, fluid])) / np.max(np.abs(ora.f))
        _say(f"   t={lat.t}: max rel err {err:.3e} ({int((~fluid).sum())} solid nodes)")
        assert err <= bound
        assert np.all(fg[:, ~fluid] == 0.0)


@pytest.mark.parametrize("nx,ny,bc,force,drag", [(61, 37, "wall", True, True), (50, 44, "periodic", True, False),
                                                  (64, 32, "wall", False, True), (130, 40, "periodic", False, True)])
def test_fused_mask_force_drag_fp64_vs_oracle(oracle, nx, ny, bc, force, drag):
    """Solid nodes with a force field and/or the drag (their own two-step
    instance, halves of 64 lanes in FP64) against the oracle."""
    torch = _torch()
    _say(f"fused mask + force={force} drag={drag} fp64 {nx}x{ny} {bc}")
    phi = field(nx, ny, nx + 3 * ny)
    mask = W.solid_mask(nx, ny, seed=nx + ny + 2)
    fluid = mask == 0
    f0 = W.random_populations(nx, ny, seed=23 + nx)
    g = (2e-5, -1e-5)
    fc = (2e-6 * W.smoothed_noise(nx, ny, 3.0, seed=31), -1e-6 * W.smoothed_noise(nx, ny, 3.0, seed=32)) if force else None
    dr = (1e-3 + 2e-2 * (1 - phi), (3e-4, -1e-4)) if drag else None
    ora = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=RATES, g=g, bc_y=bc, mask=mask, force=fc, drag=dr)
    ora.set_populations(f0)
    lat = lattice(nx, ny, phi, mask, "f64", bc, g=g, force=fc, drag=dr)
    assert lat.fused_tiling()["active"]
    lat.set_populations(torch.from_numpy(f0))
    for n, bound in ((2, 1e-14), (4, 1e-13)):
        ora.step(n)
        lat.step(n)
        fg = lat.read_populations().cpu().numpy()
        err = np.max(np.abs(fg[:, fluid] - ora.f[:, fluid])) / np.max(np.abs(ora.f))
        _say(f"   t={lat.t}: max rel err {err:.3e}")
        assert err <= bound
        assert np.all(fg[:, ~fluid] == 0.0)


@pytest.mark.parametrize("prec,nx,ny,bc,rows,drag", [
    ("f32s", 253, 130, "wall", 0, False), ("f32s", 300, 70, "periodic", 5, False),
    ("f32s", 1000, 37, "wall", 3, False), ("f32s", 246, 20, "wall", 0, False),
    ("f32s", 253, 60, "wall", 0, True), ("f32s", 130, 67, "periodic", 2, True),
    ("f16s", 253, 130, "wall", 0, False), ("f16s", 200, 50, "periodic", 0, True),
    ("f32", 97, 40, "wall", 0, False)])
def test_fused_mask_matches_single_steps(prec, nx, ny, bc, rows, drag):
    """Reduced precision: two steps per launch against one step per launch
    on the fluid nodes; solid nodes bitwise the rest state in both."""
    torch = _torch()
    _say(f"fused mask vs single {prec} {nx}x{ny} {bc} rows={rows} drag={drag}")
    phi = field(nx, ny, nx + ny)
    mask = W.solid_mask(nx, ny, seed=3 * nx + ny)
    fluid = mask == 0
    dr = (1e-3 + 0.2 * W.smoothed_noise(nx, ny, 2.0, seed=ny) ** 2, (2e-4, 0.0)) if drag else None
    f0n = W.random_populations(nx, ny, seed=29 + nx)
    f0n[:, ~fluid] = 0.0
    f0 = torch.from_numpy(f0n)
    a = lattice(nx, ny, phi, mask, prec, bc, fused=False, drag=dr)
    b = lattice(nx, ny, phi, mask, prec, bc, fused=True, rows=rows, drag=dr)
    assert b.fused_tiling()["active"] and not a.fused_tiling()["active"]
    a.set_populations(f0)
    b.set_populations(f0)
    bound = {"f32s": FUSED_RTOL, "f32": FUSED_RTOL, "f16s": FUSED_RTOL16}[prec]
    for n in (2, 5, 4):
        a.step(n)
        b.step(n)
        fa = a.read_populations().cpu().numpy()
        fb = b.read_populations().cpu().numpy()
        rel = fluid_rel_diff(fa, fb, f0n, fluid)
        _say(f"  after {a.t} steps: fluid relative difference {rel:.3e}")
        assert rel <= bound, (n, rel)
        assert np.array_equal(fa[:, ~fluid], fb[:, ~fluid])


def _cylinder(nx=96, ny=40):
    phi = W.channel_phi(nx, ny, seed=11, lo=0.6)
    return phi, W.cylinder_channel(nx, ny, radius=6.0)


def test_fused_cylinder_channel_fp64(oracle):
    """Flow past a cylinder between walls, 800 steps with two steps per
    launch, against the oracle: rel-L2(u) <= 1e-12 on fluid nodes, mass
    conserved and equal to the oracle's."""
    _torch()
    nx, ny, steps = 96, 40, 800
    phi, mask = _cylinder(nx, ny)
    fluid = mask == 0
    ora = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=RATES, g=(2e-6, 0), bc_y="wall",
                        mask=mask).init_equilibrium()
    ora.step(steps)
    ref = ora.macroscopic()
    lat = lattice(nx, ny, phi, mask, "f64", "wall", g=(2e-6, 0))
    lat.init_equilibrium(1.0)
    obs0 = lat.observe()
    lat.step(steps)
    m = {k: v.cpu().numpy() for k, v in lat.read_moments().items()}
    e = rel_l2_u(m, ref, fluid)
    obs = lat.observe()
    mass_ref = float(np.sum(ora.f[:, fluid]))
    _say(f"fused cylinder fp64: rel-L2(u) {e:.3e}, mass {obs['mass']:.15e} vs {mass_ref:.15e}")
    assert e <= 1e-12
    assert abs(obs["mass"] - mass_ref) <= 1e-13 * mass_ref
    assert abs(obs["mass"] - obs0["mass"]) <= 1e-13 * obs0["mass"]
    assert np.all(m["ux"][~fluid] == 0.0)


@pytest.mark.parametrize("prec,bound", [("f32s", 1e-4), ("f16s", 5e-2)])
def test_fused_cylinder_reduced_precision(oracle, prec, bound):
    """The same bounds as one step per launch."""
    _torch()
    nx, ny, steps = 96, 40, 400
    phi, mask = _cylinder(nx, ny)
    fluid = mask == 0
    ora = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=RATES, g=(2e-6, 0), bc_y="wall",
                        mask=mask).init_equilibrium()
    ora.step(steps)
    ref = ora.macroscopic()
    lat = lattice(nx, ny, phi, mask, prec, "wall", g=(2e-6, 0))
    lat.init_equilibrium(1.0).step(steps)
    e = rel_l2_u({k: v.cpu().numpy() for k, v in lat.read_moments().items()}, ref, fluid)
    _say(f"fused cylinder {prec}: rel-L2(u) {e:.3e}")
    assert e <= bound


@pytest.mark.parametrize("precision,drag,threads", [("f32s", False, 256), ("f32s", False, 64),
                                                    ("f64", False, 128), ("f16s", True, 128),
                                                    ("f32s", True, 64), ("f64", True, 64)])
def test_two_step_batch_with_masks(precision, drag, threads):
    """Members with solid nodes (and the drag): bitwise the results of
    stepping each member alone with two steps per launch, odd last step
    included."""
    _torch()
    from paper_2409_02964_amd.vanse import Batch
    sizes = [(64, 48), (37, 53), (130, 20), (300, 31), (17, 5)]

    def member(k, nx, ny):
        phi = 0.6 + 0.3 * np.sin(2 * np.pi * np.arange(nx)[None, :] / nx) * np.cos(2 * np.pi * np.arange(ny)[:, None] / ny)
        dr = (1e-3 + 2e-2 * (1 - phi), (1e-4 * k, 0.0)) if drag else None
        lat = lattice(nx, ny, phi, W.solid_mask(nx, ny, seed=40 + k), precision, "wall", fused=True,
                      g=(1e-6 * (k + 1), 0.0), drag=dr)
        return lat.init_equilibrium(1.0, 1e-3, 0.0)

    ref = [member(k, nx, ny) for k, (nx, ny) in enumerate(sizes)]
    for lat in ref:
        assert lat.fused_tiling()["active"]
        lat.step(11)
    mem = [member(k, nx, ny) for k, (nx, ny) in enumerate(sizes)]
    Batch(mem, threads=threads, rows=7, graph_steps=4, steps_per_pass=2).step(11)
    for a, r in zip(mem, ref):
        assert a.t == r.t == 11
        assert np.array_equal(a.read_populations().cpu().numpy(), r.read_populations().cpu().numpy())


def test_two_step_mask_widths_and_fallbacks():
    """Solid nodes with the drag take halves of at most 128 lanes in FP32
    arithmetic and 64 in FP64 (alone: 256 and 128, as without solid nodes);
    walls in x still take one step per launch."""
    torch = _torch()
    from paper_2409_02964_amd.vanse import Batch, Lattice, VanseError
    n = 48
    phi = W.periodic_wave(n, n)
    mask = W.solid_mask(n, n, seed=1)
    Batch([lattice(n, n, phi, mask, "f32s").init_equilibrium(1.0)], threads=256, steps_per_pass=2).step(2)
    f32 = [lattice(n, n, phi, mask, "f32s", drag=(np.full((n, n), 1e-3), (0.0, 0.0))).init_equilibrium(1.0)]
    with pytest.raises(VanseError):
        Batch(f32, threads=256, steps_per_pass=2)
    Batch(f32, threads=128, steps_per_pass=2).step(2)
    f64 = [lattice(n, n, phi, mask, "f64", drag=(np.full((n, n), 1e-3), (0.0, 0.0))).init_equilibrium(1.0)]
    with pytest.raises(VanseError):
        Batch(f64, threads=128, steps_per_pass=2)
    Batch(f64, threads=64, steps_per_pass=2).step(2)
    a = Lattice(n, n, "f32", bc_x="wall", bc_y="wall")
    b = Lattice(n, n, "f32", bc_x="wall", bc_y="wall")
    for lat in (a, b):
        lat.set_params(0.5, RATES).set_body_force(1e-6, 0).set_void_fraction(phi)
    b.set_steps_per_pass(2)
    assert not b.fused_tiling()["active"]  # walls in x: one step per launch
    for lat in (a, b):
        lat.init_equilibrium(1.0)
        lat.step(7)
    assert torch.equal(a.read_populations(), b.read_populations())


# ---- the scheme variants with solid nodes: model B (Sec. 2.3: kappa - 1 for
# kappa - phi, the solid-neighbour terms of the penalty included) and the
# Appendix B equilibrium (the penalty of Eq. B3) ------------------------------

SCHEMES = {"B": ("B", 3), "AppB": ("A", 2), "B+AppB": ("B", 2)}


@pytest.mark.parametrize("scheme", ["B", "AppB", "B+AppB"])
@pytest.mark.parametrize("nx,ny,bc,rows,force,drag", [
    (61, 37, "wall", 0, False, False), (64, 48, "periodic", 3, False, False),
    (130, 40, "wall", 0, True, True), (50, 44, "periodic", 1, False, True)])
def test_fused_mask_scheme_fp64_vs_oracle(oracle, scheme, nx, ny, bc, rows, force, drag):
    """A scheme variant with solid nodes, two steps per launch in FP64 (with
    the force field and drag or not), node by node against the FP64 oracle."""
    torch = _torch()
    model, order = SCHEMES[scheme]
    _say(f"fused mask {scheme} fp64 vs oracle {nx}x{ny} {bc} rows={rows} force={force} drag={drag}")
    phi = field(nx, ny, nx + 5 * ny)
    mask = W.solid_mask(nx, ny, seed=nx * ny + 3)
    fluid = mask == 0
    f0 = W.random_populations(nx, ny, seed=23 + nx)
    g = (2e-5, -1e-5)
    fc = (1e-5 * W.smoothed_noise(nx, ny, 3.0, seed=1), -1e-5 * W.smoothed_noise(nx, ny, 3.0, seed=2)) if force else None
    dr = (1e-3 + 0.1 * W.smoothed_noise(nx, ny, 2.0, seed=ny) ** 2, (1e-4, 0.0)) if drag else None
    ora = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=RATES, g=g, bc_y=bc, mask=mask, model_b=model == "B",
                        eq2=order == 2, force=fc, drag=dr)
    ora.set_populations(f0)
    lat = lattice(nx, ny, phi, mask, "f64", bc, rows=rows, g=g, force=fc, drag=dr)
    lat.set_scheme(model, order)
    assert lat.fused_tiling()["active"]
    lat.set_populations(torch.from_numpy(f0))
    for n, bound in ((2, 1e-14), (5, 1e-13)):
        ora.step(n)
        lat.step(n)
        fg = lat.read_populations().cpu().numpy()
        err = np.max(np.abs(fg[:, fluid] - ora.f[:, fluid])) / np.max(np.abs(ora.f))
        _say(f"   t={lat.t}: max rel err {err:.3e}")
        assert err <= bound
        assert np.all(fg[:, ~fluid] == 0.0)


@pytest.mark.parametrize("scheme", ["B", "AppB"])
def test_fused_mask_scheme_matches_single_steps(scheme):
    """A scheme variant with solid nodes in FP32-shifted storage: two steps
    per launch against one (the instance with every input), to FP32
    rounding."""
    torch = _torch()
    model, order = SCHEMES[scheme]
    nx, ny = 253, 130
    phi = field(nx, ny, 11)
    mask = W.solid_mask(nx, ny, seed=17)
    fluid = mask == 0
    f0 = W.random_populations(nx, ny, seed=29)
    f0[:, ~fluid] = 0.0
    a = lattice(nx, ny, phi, mask, "f32s", "wall", fused=False)
    b = lattice(nx, ny, phi, mask, "f32s", "wall", fused=True)
    for lat in (a, b):
        lat.set_scheme(model, order)
        lat.set_populations(torch.from_numpy(f0))
    assert b.fused_tiling()["active"] and not a.fused_tiling()["active"]
    for n in (2, 5, 4):
        a.step(n)
        b.step(n)
    rel = fluid_rel_diff(a.read_populations().cpu().numpy(), b.read_populations().cpu().numpy(), f0, fluid)
    _say(f"{scheme} with solid nodes, two steps vs one: relative difference {rel:.3e}")
    assert rel <= 1e-5
