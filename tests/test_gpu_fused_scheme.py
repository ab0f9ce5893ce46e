"""Two time steps per launch for the scheme variants: model B (Sec. 2.3:
kappa - 1 in place of kappa - phi in F^p and in the source term of Eq. 20)
and the Appendix B equilibrium (B1, B2, and the penalty of Eq. B3 with twelve
derivatives), alone or combined.

The two-step kernel takes them with or without the force field and the drag
(no wall velocities, solid nodes or moving phi).  Against one step per launch
they differ by the FP32 roundings of the separable stencil sums, as the
model A kernel does (FUSED_RTOL of the two-step tests); FP64 is checked
against the FP64 oracle.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2409_02964_amd import workloads as W  # noqa: E402

RATES = dict(s_c=1.2, s_e=1.2, s_eps=1.2, s_q=1.2, s_nu=0.8)
FUSED_RTOL = 1e-5     # see the two-step tests
FUSED_RTOL64 = 1e-12


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def lattice(nx, ny, phi, precision, bc, spp, rows=0, g=(2e-5, -1e-5), drag=None, force=None, order=3,
            wall_u=None, model="B"):
    from paper_2409_02964_amd.vanse import Lattice
    lat = Lattice(nx, ny, precision=precision, bc_y=bc, drag=drag is not None,
                  force_field=force is not None)
    lat.set_params(0.5, RATES).set_body_force(*g).set_scheme(model, order)
    if wall_u is not None:
        lat.set_wall_velocity(*wall_u)
    lat.set_void_fraction(phi)
    if drag is not None:
        lat.set_drag(drag)
    if force is not None:
        lat.set_force_field(*force)
    lat.set_steps_per_pass(spp, rows)
    return lat


def rel_diff(fa, fb, f0):
    return float(abs(fa - fb).max() / abs(fa - f0).max())


def rel_l2_u(m, ref):
    num = np.sum((m["ux"] - ref["ux"]) ** 2 + (m["uy"] - ref["uy"]) ** 2)
    return math.sqrt(num / np.sum(ref["ux"] ** 2 + ref["uy"] ** 2))


SCHEMES = {"B": ("B", 3), "AppB": ("A", 2), "B+AppB": ("B", 2)}


@pytest.mark.parametrize("scheme", ["B", "AppB", "B+AppB"])
@pytest.mark.parametrize("prec,bc,nx,ny,rows,drag,force", [
    ("f32s", "wall", 253, 130, 0, False, False), ("f32s", "periodic", 300, 70, 7, False, False),
    ("f32s", "wall", 97, 2, 0, False, False), ("f32s", "wall", 1000, 37, 5, True, False),
    ("f32s", "periodic", 130, 67, 1, False, True), ("f32s", "wall", 246, 60, 0, True, True),
    ("f64", "wall", 253, 130, 0, False, False), ("f64", "periodic", 130, 67, 3, True, True)])
def test_scheme_two_steps_match_single_steps(scheme, prec, bc, nx, ny, rows, drag, force):
    torch = _torch()
    _say(f"{scheme} two steps vs one {prec} {nx}x{ny} {bc} rows={rows} drag={drag} force={force}")
    phi = 0.55 + 0.4 * W.smoothed_noise(nx, ny, 2.0, seed=nx + ny) ** 2
    beta = (1e-3 + 0.2 * W.smoothed_noise(nx, ny, 2.0, seed=ny) ** 2) if drag else None
    ff = ((1e-5 * W.smoothed_noise(nx, ny, 3.0, seed=1), -1e-5 * W.smoothed_noise(nx, ny, 3.0, seed=2))
          if force else None)
    f0n = W.random_populations(nx, ny, seed=19 + nx)
    f0 = torch.from_numpy(f0n)
    model, order = SCHEMES[scheme]
    a = lattice(nx, ny, phi, prec, bc, 1, drag=beta, force=ff, model=model, order=order)
    b = lattice(nx, ny, phi, prec, bc, 2, rows=rows, drag=beta, force=ff, model=model, order=order)
    assert b.fused_tiling()["active"] and not a.fused_tiling()["active"]
    a.set_populations(f0)
    b.set_populations(f0)
    for n in (2, 5, 1, 4):
        a.step(n)
        b.step(n)
        rel = rel_diff(a.read_populations().cpu().numpy(), b.read_populations().cpu().numpy(), f0n)
        _say(f"  after {a.t} steps: relative difference {rel:.3e}")
        assert a.t == b.t
        assert rel <= (FUSED_RTOL64 if prec == "f64" else FUSED_RTOL), (n, rel)


@pytest.mark.parametrize("scheme,drag", [("B", False), ("B", True), ("AppB", False), ("AppB", True),
                                         ("B+AppB", False)])
def test_scheme_two_steps_fp64_vs_oracle(oracle, scheme, drag):
    """The scheme variants with two steps per launch in FP64, a walled
    channel, against the FP64 oracle at rel-L2(u) <= 1e-12."""
    _torch()
    model, order = SCHEMES[scheme]
    nx, ny, steps = 64, 48, 400
    phi = W.channel_phi(nx, ny, seed=3, lo=0.5)
    beta = (2e-3 + 1e-2 * (1 - phi)) if drag else None
    g = (2e-6, 0)
    ora = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=RATES, g=g, bc_y="wall", model_b=model == "B",
                        eq2=order == 2, drag=None if beta is None else (beta, (0.0, 0.0))).init_equilibrium()
    ora.step(steps)
    lat = lattice(nx, ny, phi, "f64", "wall", 2, g=g, drag=beta, model=model, order=order)
    assert lat.fused_tiling()["active"]
    lat.init_equilibrium(1.0).step(steps)
    m = {k: v.cpu().numpy() for k, v in lat.read_moments().items()}
    err = rel_l2_u(m, ora.macroscopic())
    _say(f"{scheme}, two steps per launch, FP64, drag={drag}: rel-L2(u) vs oracle {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("scheme", ["B", "AppB"])
def test_scheme_two_step_batch_is_bitwise_the_members(scheme):
    """A batch of lattices of one scheme variant with two steps per launch
    gives, bitwise, each member stepped alone with two steps per launch (an
    odd count ends with one step of each)."""
    _torch()
    model, order = SCHEMES[scheme]
    from paper_2409_02964_amd.vanse import Batch
    sizes = [(64, 48), (37, 53), (130, 20), (90, 31)]

    def member(k, nx, ny):
        phi = 0.6 + 0.3 * np.sin(2 * np.pi * np.arange(nx)[None, :] / nx) * np.cos(2 * np.pi * np.arange(ny)[:, None] / ny)
        lat = lattice(nx, ny, phi, "f32s", "wall", 2, g=(1e-6 * (k + 1), 0.0),
                      drag=1e-3 + 2e-2 * (1 - phi), model=model, order=order)
        return lat.init_equilibrium(1.0, 1e-3, 0.0)

    ref = [member(k, nx, ny) for k, (nx, ny) in enumerate(sizes)]
    for lat in ref:
        assert lat.fused_tiling()["active"]
        lat.step(11)
    mem = [member(k, nx, ny) for k, (nx, ny) in enumerate(sizes)]
    Batch(mem, threads=128, rows=7, graph_steps=0, steps_per_pass=2).step(11)
    for a, r in zip(mem, ref):
        assert a.t == r.t == 11
        assert np.array_equal(a.read_populations().cpu().numpy(), r.read_populations().cpu().numpy())


@pytest.mark.parametrize("case", ["wall_velocity", "wall_velocity_appendix_b"])
def test_wall_velocities_keep_one_step(case):
    """Wall velocities stay with one step per launch even when two are asked
    for, and step bitwise as without."""
    torch = _torch()
    nx, ny = 60, 30
    phi = 0.55 + 0.4 * W.smoothed_noise(nx, ny, 2.0, seed=5) ** 2
    kw = dict(wall_u=(0.0, 1e-3), order=2 if case.endswith("appendix_b") else 3)
    a = lattice(nx, ny, phi, "f32s", "wall", 1, **kw)
    b = lattice(nx, ny, phi, "f32s", "wall", 2, **kw)
    assert not b.fused_tiling()["active"]
    for lat in (a, b):
        lat.init_equilibrium(1.0).step(7)
    assert torch.equal(a.read_populations(), b.read_populations())
