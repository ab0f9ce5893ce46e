"""Two time steps per launch (vanse_set_steps_per_pass(2)).

The two-step kernel runs the scheme twice per pass with the intermediate
populations kept as FP32 deviations in LDS.  With FP32-shifted storage that
is what one step per launch stores and loads; the two kernels differ only in
the order of the FP32 sums of the Eq. (10) stencils (the two-step kernel
uses the stencil's separable form), so they agree to FP32 rounding
(FUSED_RTOL below).  Plain FP32 and FP16-shifted storage also skip one
storage rounding per pair and are checked against the FP64 oracle.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2409_02964_amd import workloads as W  # noqa: E402

RATES = dict(s_c=1.2, s_e=1.2, s_eps=1.2, s_q=1.2, s_nu=0.8)


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def lattice(nx, ny, phi, precision, bc, fused, rows=0, g=(2e-5, -1e-5), drag=None, force=None):
    from paper_2409_02964_amd.vanse import Lattice
    lat = Lattice(nx, ny, precision=precision, bc_y=bc, drag=drag is not None,
                  force_field=force is not None)
    lat.set_params(0.5, RATES).set_body_force(*g).set_void_fraction(phi)
    if drag is not None:
        lat.set_drag(drag)
    if force is not None:
        lat.set_force_field(*force)
    if fused:
        lat.set_steps_per_pass(2, rows)
    return lat


# The two kernels round the stencil sums differently: a few FP32 ulps (6e-8
# relative) of the penalty and force terms per step, which the collision (a
# contraction, |1 - s| < 1) does not amplify.  Measured against how far the
# state moved (max |f(t) - f(0)|), the difference after the dozen steps
# compared here stays below 5e-7; 1e-5 leaves a twentyfold margin, while a
# wrong ring row, lane or wall image is an error of the size of the change
# itself.
FUSED_RTOL = 1e-5


def fused_rel_diff(fa, fb, f0):
    """max |fa - fb| / max |fa - f0| (numpy or torch)"""
    return float(abs(fa - fb).max() / abs(fa - f0).max())


def rel_l2_u(m, ref):
    num = np.sum((m["ux"] - ref["ux"]) ** 2 + (m["uy"] - ref["uy"]) ** 2)
    return math.sqrt(num / np.sum(ref["ux"] ** 2 + ref["uy"] ** 2))


SHAPES = [
    (300, 70, "periodic", 0),
    (253, 130, "wall", 0),
    (64, 64, "periodic", 0),
    (97, 2, "wall", 0),      # both walls on every row
    (1000, 37, "wall", 5),   # many strips and row blocks, ragged tails
    (247, 33, "periodic", 4),
    (246, 20, "wall", 3),    # exactly one strip
    (3, 5, "periodic", 0),   # everything wraps
    (253, 130, "wall", 1),   # one row per workgroup: every row a block edge
    (130, 67, "periodic", 2),
]


@pytest.mark.parametrize("nx,ny,bc,rows", SHAPES)
def test_fused_matches_single_steps_f32s(nx, ny, bc, rows):
    torch = _torch()
    _say(f"fused vs single f32s {nx}x{ny} {bc} rows={rows}")
    phi = 0.55 + 0.4 * W.smoothed_noise(nx, ny, 2.0, seed=nx + ny) ** 2
    f0n = W.random_populations(nx, ny, seed=7 + nx)
    f0 = torch.from_numpy(f0n)
    a = lattice(nx, ny, phi, "f32s", bc, fused=False)
    b = lattice(nx, ny, phi, "f32s", bc, fused=True, rows=rows)
    assert b.fused_tiling()["active"] and not a.fused_tiling()["active"]
    a.set_populations(f0)
    b.set_populations(f0)
    for n in (2, 5, 1, 4):  # pairs, a pair plus a single step, ...
        a.step(n)
        b.step(n)
        fa = a.read_populations().cpu().numpy()
        fb = b.read_populations().cpu().numpy()
        assert a.t == b.t
        rel = fused_rel_diff(fa, fb, f0n)
        _say(f"  after {a.t} steps: max |f_fused - f_single| / max |f - f0| = {rel:.3e}")
        assert rel <= FUSED_RTOL, (n, rel)


@pytest.mark.parametrize("prec,bound", [("f32", 5e-2), ("f16s", 5e-2)])
def test_fused_periodic_wave_vs_oracle(oracle, prec, bound):
    _torch()
    n, steps = 64, 1000
    phi = W.periodic_wave(n, n)
    ora = oracle.Oracle(n, n, phi, kappa=0.5, rates=RATES, g=(1e-6, 0)).init_equilibrium()
    ora.step(steps)
    ref = ora.macroscopic()
    single = lattice(n, n, phi, prec, "periodic", fused=False, g=(1e-6, 0))
    fused = lattice(n, n, phi, prec, "periodic", fused=True, g=(1e-6, 0))
    out = {}
    for name, lat in (("single", single), ("fused", fused)):
        lat.init_equilibrium(1.0)
        lat.step(steps)
        out[name] = {k: v.cpu().numpy() for k, v in lat.read_moments().items()}
    e_s, e_f = rel_l2_u(out["single"], ref), rel_l2_u(out["fused"], ref)
    _say(f"periodic wave {prec}: rel-L2(u) single {e_s:.3e}, fused {e_f:.3e}")
    assert e_f <= bound
    assert e_f <= 1.5 * e_s + 1e-6  # one storage rounding fewer per pair: not worse


def test_fused_full_size_channel():
    """The 4096 x 4096 channel (walls, the benchmark field) in FP32-shifted
    storage: three two-step launches and six single steps agree to FP32
    rounding."""
    torch = _torch()
    n = 4096
    phi = W.channel_phi(n, n, seed=2409)
    a = lattice(n, n, phi, "f32s", "wall", fused=False, g=(1e-7, 0))
    b = lattice(n, n, phi, "f32s", "wall", fused=True, g=(1e-7, 0))
    for lat in (a, b):
        lat.init_equilibrium(1.0)
    f0 = a.read_populations()
    for lat in (a, b):
        lat.step(6)
    fa, fb = a.read_populations(), b.read_populations()
    rel = fused_rel_diff(fa, fb, f0)
    _say(f"full-size fused vs single: relative diff {rel:.3e}; fused tiling {b.fused_tiling()}")
    assert rel <= FUSED_RTOL
    a.close()
    b.close()


@pytest.mark.parametrize("prec,bc,nx,ny,rows", [
    ("f32s", "wall", 253, 130, 0), ("f32s", "periodic", 300, 70, 7), ("f16s", "wall", 97, 40, 0),
    ("f32", "periodic", 64, 64, 3)])
def test_fused_drag_matches_single_steps(prec, bc, nx, ny, rows):
    """The linear drag (u solved in closed form) with two steps per launch
    against one step per launch, to FP32 rounding; FP16-shifted storage
    against the single steps' own FP16 result."""
    torch = _torch()
    _say(f"fused drag vs single {prec} {nx}x{ny} {bc} rows={rows}")
    phi = 0.55 + 0.4 * W.smoothed_noise(nx, ny, 2.0, seed=nx + ny) ** 2
    beta = 1e-3 + 0.2 * W.smoothed_noise(nx, ny, 2.0, seed=ny) ** 2
    f0n = W.random_populations(nx, ny, seed=11 + nx)
    f0 = torch.from_numpy(f0n)
    a = lattice(nx, ny, phi, prec, bc, fused=False, drag=beta)
    b = lattice(nx, ny, phi, prec, bc, fused=True, rows=rows, drag=beta)
    assert b.fused_tiling()["active"] and not a.fused_tiling()["active"]
    a.set_populations(f0)
    b.set_populations(f0)
    for n in (2, 5, 4):
        a.step(n)
        b.step(n)
    fa = a.read_populations().cpu().numpy()
    fb = b.read_populations().cpu().numpy()
    rel = fused_rel_diff(fa, fb, f0n)
    _say(f"  after {a.t} steps: relative difference {rel:.3e}")
    # FP16 storage rounds each stored deviation to 11 significant bits
    # (2^-11 = 4.9e-4 relative) and the two paths store at different steps
    # (one storage rounding fewer per pair): the difference is about one such
    # rounding of the change (3.4e-4 measured); 2e-3 allows four
    assert rel <= (FUSED_RTOL if prec != "f16s" else 2e-3)


def test_fused_falls_back_for_variants():
    torch = _torch()
    from paper_2409_02964_amd.vanse import Lattice, VanseError
    n = 48
    phi = W.periodic_wave(n, n)
    a = Lattice(n, n, "f32", bc_x="wall")
    b = Lattice(n, n, "f32", bc_x="wall")
    for lat in (a, b):
        lat.set_params(0.5, RATES).set_body_force(1e-6, 0).set_void_fraction(phi)
    b.set_steps_per_pass(2)
    assert not b.fused_tiling()["active"]  # walls in x: one step per launch
    for lat in (a, b):
        lat.init_equilibrium(1.0)
        lat.step(7)
    assert torch.equal(a.read_populations(), b.read_populations())
    with pytest.raises(VanseError):
        a.set_steps_per_pass(3)


# ---- FP64: halves of 128 lanes, the same scheme in double ---------------------------

# The FP64 two-step kernel orders the Eq. (10) sums as the FP32 one does, so
# against FP64 single steps it differs by FP64 roundings (1.1e-16 relative)
# of the penalty and force terms; measured against the state change as above
# that is below 1e-15 (7e-16 on these shapes).  1e-12 leaves a wide margin
# and still flags a wrong ring row, lane or wall image, an error of the size
# of the change.
FUSED_RTOL64 = 1e-12


@pytest.mark.parametrize("nx,ny,bc,rows,drag", [
    (300, 70, "periodic", 0, False), (253, 130, "wall", 0, False), (97, 2, "wall", 0, False),
    (1000, 37, "wall", 5, False), (3, 5, "periodic", 0, False), (253, 130, "wall", 1, False),
    (246, 60, "wall", 0, True), (130, 67, "periodic", 3, True)])
def test_fused_fp64_matches_single_steps(nx, ny, bc, rows, drag):
    torch = _torch()
    _say(f"fused vs single f64 {nx}x{ny} {bc} rows={rows} drag={drag}")
    phi = 0.55 + 0.4 * W.smoothed_noise(nx, ny, 2.0, seed=nx + ny) ** 2
    beta = (1e-3 + 0.2 * W.smoothed_noise(nx, ny, 2.0, seed=ny) ** 2) if drag else None
    f0n = W.random_populations(nx, ny, seed=13 + nx)
    f0 = torch.from_numpy(f0n)
    a = lattice(nx, ny, phi, "f64", bc, fused=False, drag=beta)
    b = lattice(nx, ny, phi, "f64", bc, fused=True, rows=rows, drag=beta)
    assert b.fused_tiling()["active"] and not a.fused_tiling()["active"]
    a.set_populations(f0)
    b.set_populations(f0)
    for n in (2, 5, 1, 4):
        a.step(n)
        b.step(n)
        fa = a.read_populations().cpu().numpy()
        fb = b.read_populations().cpu().numpy()
        assert a.t == b.t
        rel = fused_rel_diff(fa, fb, f0n)
        _say(f"  after {a.t} steps: max |f_fused - f_single| / max |f - f0| = {rel:.3e}")
        assert rel <= FUSED_RTOL64, (n, rel)


@pytest.mark.parametrize("bc,drag,steps", [("periodic", False, 1000), ("wall", True, 400)])
def test_fused_fp64_vs_oracle(oracle, bc, drag, steps):
    """Two steps per launch in FP64 against the FP64 oracle at the FP64
    parity bar, rel-L2(u) <= 1e-12: the periodic wave and a walled channel
    with drag."""
    _torch()
    n = 64 if bc == "periodic" else 80
    phi = W.periodic_wave(n, n) if bc == "periodic" else W.channel_phi(n, n, seed=5)
    beta = (2e-3 + 1e-2 * (1 - phi)) if drag else None
    g = (1e-6, 0)
    ora = oracle.Oracle(n, n, phi, kappa=0.5, rates=RATES, g=g, bc_y=bc,
                        drag=None if beta is None else (beta, (0.0, 0.0))).init_equilibrium()
    ora.step(steps)
    ref = ora.macroscopic()
    lat = lattice(n, n, phi, "f64", bc, fused=True, g=g, drag=beta)
    assert lat.fused_tiling()["active"]
    lat.init_equilibrium(1.0).step(steps)
    m = {k: v.cpu().numpy() for k, v in lat.read_moments().items()}
    err = rel_l2_u(m, ref)
    _say(f"f64 two steps per launch, {bc}, drag={drag}: rel-L2(u) vs oracle {err:.3e}")
    assert err <= 1e-12


# ---- the per-node force field (added to F^B in stage B) ----------------------------

@pytest.mark.parametrize("prec,bc,nx,ny,rows,drag", [
    ("f32s", "wall", 253, 130, 0, False), ("f32s", "periodic", 300, 70, 1, True),
    ("f16s", "wall", 97, 40, 0, False), ("f64", "wall", 246, 60, 0, True),
    ("f64", "periodic", 130, 67, 3, False)])
def test_fused_force_field_matches_single_steps(prec, bc, nx, ny, rows, drag):
    """A per-node force field with two steps per launch against one step per
    launch, to rounding (FP32-shifted and FP64; FP16-shifted as for the drag)."""
    torch = _torch()
    _say(f"fused force field vs single {prec} {nx}x{ny} {bc} rows={rows} drag={drag}")
    phi = 0.55 + 0.4 * W.smoothed_noise(nx, ny, 2.0, seed=nx + ny) ** 2
    force = (1e-5 * W.smoothed_noise(nx, ny, 3.0, seed=1), -1e-5 * W.smoothed_noise(nx, ny, 3.0, seed=2))
    beta = (1e-3 + 0.2 * W.smoothed_noise(nx, ny, 2.0, seed=ny) ** 2) if drag else None
    f0n = W.random_populations(nx, ny, seed=17 + nx)
    f0 = torch.from_numpy(f0n)
    a = lattice(nx, ny, phi, prec, bc, fused=False, drag=beta, force=force)
    b = lattice(nx, ny, phi, prec, bc, fused=True, rows=rows, drag=beta, force=force)
    assert b.fused_tiling()["active"] and not a.fused_tiling()["active"]
    a.set_populations(f0)
    b.set_populations(f0)
    for n in (2, 5, 4):
        a.step(n)
        b.step(n)
    rel = fused_rel_diff(a.read_populations().cpu().numpy(), b.read_populations().cpu().numpy(), f0n)
    _say(f"  after {a.t} steps: relative difference {rel:.3e}")
    bound = {"f32s": FUSED_RTOL, "f16s": 2e-3, "f64": FUSED_RTOL64}[prec]
    assert rel <= bound


def test_fused_force_field_fp64_vs_oracle(oracle):
    """FP64, two steps per launch, a per-node force field on a walled channel
    against the FP64 oracle at rel-L2(u) <= 1e-12."""
    _torch()
    n, steps = 72, 400
    phi = W.channel_phi(n, n, seed=6)
    force = (2e-6 * W.smoothed_noise(n, n, 3.0, seed=3), 1e-6 * W.smoothed_noise(n, n, 3.0, seed=4))
    g = (1e-6, 0)
    ora = oracle.Oracle(n, n, phi, kappa=0.5, rates=RATES, g=g, bc_y="wall",
                        force=force).init_equilibrium()
    ora.step(steps)
    ref = ora.macroscopic()
    lat = lattice(n, n, phi, "f64", "wall", fused=True, g=g, force=force)
    assert lat.fused_tiling()["active"]
    lat.init_equilibrium(1.0).step(steps)
    m = {k: v.cpu().numpy() for k, v in lat.read_moments().items()}
    err = rel_l2_u(m, ref)
    _say(f"f64 two steps per launch with a force field: rel-L2(u) vs oracle {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("with_mask", [False, True])
def test_fused_result_does_not_depend_on_row_tiling(with_mask):
    """The kernels are built with multiply-add fusion inside an expression
    only, so every unrolled copy of the sweep rounds a node alike: row
    tilings of the two-step kernel agree bitwise (random populations, walls,
    ten steps; solid nodes or none)."""
    torch = _torch()
    from paper_2409_02964_amd.vanse import Lattice
    nx, ny = 253, 130
    phi = 0.55 + 0.4 * W.smoothed_noise(nx, ny, 2.0, seed=nx + ny) ** 2
    mask = W.solid_mask(nx, ny, seed=3) if with_mask else None
    f0 = W.random_populations(nx, ny, seed=7 + nx)
    if with_mask:
        f0[:, mask != 0] = 0.0
    out = {}
    for rows in (0, 5, 6, 7, 13, 40):
        lat = Lattice(nx, ny, precision="f32s", bc_y="wall", mask=with_mask)
        lat.set_params(0.5, RATES).set_body_force(2e-5, -1e-5)
        if with_mask:
            lat.set_mask(mask)
        lat.set_void_fraction(phi).set_steps_per_pass(2, rows)
        lat.set_populations(torch.from_numpy(f0))
        lat.step(10)
        out[rows] = lat.read_populations().cpu().numpy()
        lat.close()
    for rows, f in out.items():
        _say(f"  rows={rows}: {int(np.sum(f != out[0]))} values differ from the default tiling")
        assert np.array_equal(f, out[0])
