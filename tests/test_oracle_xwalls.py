"""Walls in x in the FP64 oracle, pinned by symmetry (CPU).

D2Q9 and the scheme are invariant under the exchange of x and y: the moment
set of Eq. A1 maps onto itself (j_x <-> j_y, q_x <-> q_y, p_xx -> -p_xx,
p_xy -> p_xy) with equal rates for each pair, and Eq. 10, Eq. 13 and Eq. 20
are isotropic.  So a lattice with walls at its x faces, run on the transposed
inputs, must reproduce the transpose of the same run with walls at its y
faces, which the channel tests (Poiseuille, solid rows) pin.  This checks the
x-wall pull, the mirror images of the stencils across x faces and the corner
where both walls meet.
"""
import numpy as np
import pytest

from paper_2409_02964_amd import workloads as W

RATES = dict(s_c=1.2, s_e=1.1, s_eps=1.3, s_q=1.15, s_nu=0.8)
# direction i of (e_x, e_y) -> direction of (e_y, e_x)
SWAP = [0, 2, 1, 4, 3, 5, 8, 7, 6]


def transpose_pops(f):
    return np.stack([f[SWAP[i]].T for i in range(9)])


@pytest.mark.parametrize("bc_other,with_mask,coupled", [("periodic", False, False),
                                                         ("wall", False, False),
                                                         ("wall", True, True),
                                                         ("periodic", True, False)])
def test_x_walls_are_transposed_y_walls(oracle, bc_other, with_mask, coupled):
    nx, ny, steps = 23, 17, 40   # the y-wall run; the x-wall run is ny x nx
    phi = 0.55 + 0.4 * W.smoothed_noise(nx, ny, 2.0, seed=3) ** 2
    mask = W.solid_mask(nx, ny, seed=4) if with_mask else None
    f0 = W.random_populations(nx, ny, seed=6)
    g = (1.5e-5, -4e-6)
    force = drag = None
    if coupled:
        force = (2e-6 * W.smoothed_noise(nx, ny, 3.0, seed=7), -1e-6 * W.smoothed_noise(nx, ny, 3.0, seed=8))
        drag = (1e-3 + 2e-2 * (1 - phi), (3e-4, -1e-4))
    a = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=RATES, g=g, bc_x=bc_other, bc_y="wall",
                      mask=mask, force=force, drag=drag)
    a.set_populations(f0)
    a.step(steps)
    b = oracle.Oracle(ny, nx, phi.T, kappa=0.5, rates=RATES, g=(g[1], g[0]), bc_x="wall",
                      bc_y=bc_other, mask=None if mask is None else mask.T.copy(),
                      force=None if force is None else (force[1].T, force[0].T),
                      drag=None if drag is None else (drag[0].T, (drag[1][1], drag[1][0])))
    b.set_populations(transpose_pops(f0))
    b.step(steps)
    scale = np.max(np.abs(a.f))
    assert np.max(np.abs(transpose_pops(a.f) - b.f)) <= 1e-13 * scale
    ma, mb = a.macroscopic(), b.macroscopic()
    assert np.max(np.abs(ma["ux"].T - mb["uy"])) <= 1e-13 * np.max(np.abs(ma["ux"]))
    assert np.max(np.abs(ma["uy"].T - mb["ux"])) <= 1e-13 * np.max(np.abs(ma["ux"]))


def test_x_wall_mistake_is_caught(oracle):
    """The symmetry check is sharp: with the x-wall run's body force left
    untransposed the populations differ by far more than rounding."""
    nx, ny = 23, 17
    phi = 0.55 + 0.4 * W.smoothed_noise(nx, ny, 2.0, seed=3) ** 2
    f0 = W.random_populations(nx, ny, seed=6)
    a = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=RATES, g=(1.5e-5, -4e-6), bc_y="wall")
    a.set_populations(f0)
    a.step(10)
    b = oracle.Oracle(ny, nx, phi.T, kappa=0.5, rates=RATES, g=(1.5e-5, -4e-6), bc_x="wall")
    b.set_populations(transpose_pops(f0))
    b.step(10)
    assert np.max(np.abs(transpose_pops(a.f) - b.f)) > 1e-9 * np.max(np.abs(a.f))
