"""Pins of the Eq. (10) stand-in next to a half-way wall (CPU).

The paper leaves open what stands in for a stencil neighbour beyond a wall;
the oracle takes the mirror image across the wall face, scalars copied and
velocity-like fields negated.  Two exact properties fix the three parts of
that reading:
  * plain Couette flow between half-way walls is the exact linear profile,
    which holds only with the velocity image negated (no slip) and taken
    across the face (y = -1/2), not across the wall row;
  * a closed box at rest under a body force along a pair of walls stays at
    rest, with a density that does not vary across the box: the stand-in of a
    diagonal neighbour must be the image of that neighbour, not the centre
    node's own value (which would give the tangential derivatives on the
    wall rows the wrong weight and drive currents along the wall).
The last test plants each of the three plausible mistakes in a copy of the
oracle's source and shows that one of these pins fails for it."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

G = 1e-5
BOX_RATES = dict(s_c=1.0, s_e=1.2, s_eps=1.2, s_q=1.2, s_nu=1.0)


def _box(oracle, phi_varies):
    """Closed 24 x 10 box (walls in x and y), F^B = phi G along x, kappa = 0.5,
    6000 steps from rest: (max |u| / G, max over rows of the spread of rho
    across y relative to G nx)."""
    nx, ny = 24, 10
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    phi = (0.6 + 0.3 * np.sin(np.pi * (x + 0.5) / nx) ** 2) if phi_varies else np.full((ny, nx), 0.7)
    o = oracle.Oracle(nx, ny, phi, kappa=0.5, rates=BOX_RATES, g=(G, 0.0), bc_x="wall",
                      bc_y="wall").init_equilibrium()
    o.step(6000)
    m = o.macroscopic()
    umax = max(np.max(np.abs(m["ux"])), np.max(np.abs(m["uy"])))
    spread = np.max(np.abs(m["rho"] - m["rho"][ny // 2][None, :]))
    return umax / G, spread / (G * nx)


@pytest.mark.parametrize("phi_varies", [False, True])
def test_box_at_rest_under_force_along_walls(oracle, phi_varies):
    """Hydrostatic equilibrium along the walls: the fluid stays at rest (to
    rounding) and rho depends on x alone, on the rows next to the y-walls as
    in the middle of the box, for phi uniform and for phi varying along x
    (kappa != phi, so F^p of Eq. 13 and the penalty terms are active)."""
    urel, spread = _box(oracle, phi_varies)
    assert urel < 1e-7
    assert spread < 1e-9


def _couette_error(oracle):
    """Couette flow, 4 x 12, phi = 0.8 (kappa = 0.5), lower wall at rest, upper
    half-way wall moving at U: max |u - U (y + 1/2) / H| / U after 8 H^2/nu
    steps (nu = 0.1)."""
    H, nx, U, nu = 12, 4, 1e-3, 0.1
    rates = dict(s_c=1.0, s_e=1.0 / (nu + 0.5), s_eps=1.2, s_q=1.4, s_nu=1.0 / (3 * nu + 0.5))
    o = oracle.Oracle(nx, H, np.full((H, nx), 0.8), kappa=0.5, rates=rates, bc_y="wall",
                      wall_velocity=(0.0, U)).init_equilibrium()
    o.step(int(8 * H * H / nu))
    u = o.macroscopic()["ux"][:, 0]
    return float(np.max(np.abs(u - U * (np.arange(H) + 0.5) / H)) / U)


# A copy of the oracle built from mutated source runs in a child process (the
# oracle module loads one library per process); it prints the pins' figures.
_CHILD = r"""
import sys
sys.path.insert(0, {root!r})
sys.path.insert(0, {tests!r})
import oracle.oracle as O
O._LIB = sys.argv[1]
import test_oracle_wall_pins as T
print(T._couette_error(O), *T._box(O, False), *T._box(O, True))
"""

# the y-wall image in the oracle's neighbour lookup, and the planted mistakes
_IMAGE = """      *wall = (yn < 0) ? 1 : 2;
      yn = (yn < 0) ? -1 - yn : 2 * P->ny - 1 - yn;
      reflected = 1;"""
_MUTANTS = {
    # velocity-like fields copied instead of negated (free slip)
    "velocity copied": """      *wall = (yn < 0) ? 1 : 2;
      yn = (yn < 0) ? -1 - yn : 2 * P->ny - 1 - yn;""",
    # the image across the wall row instead of the wall face
    "image across the wall row": """      *wall = (yn < 0) ? 1 : 2;
      yn = (yn < 0) ? -yn : 2 * P->ny - 2 - yn;
      reflected = 1;""",
    # the centre node's own value (as for a solid neighbour)
    "centre value": """      *wall = (yn < 0) ? 1 : 2;
      yn = y; xn = x;
      reflected = 1;""",
}


def _pins_with(source, tmp_path, name):
    cc = shutil.which("gcc")
    lib = str(tmp_path / f"lib_{name}.so")
    src = str(tmp_path / f"{name}.c")
    with open(src, "w") as fh:
        fh.write(source)
    subprocess.run([cc, "-O3", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-o", lib, src, "-lm"], check=True, capture_output=True, timeout=300)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", _CHILD.format(root=ROOT, tests=HERE), lib],
                         check=True, capture_output=True, text=True, timeout=600, env=env)
    couette, u0, s0, u1, s1 = (float(v) for v in out.stdout.split())
    return couette, max(u0, u1), max(s0, s1)


def test_wall_pins_catch_planted_mistakes(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    with open(os.path.join(ROOT, "oracle", "vanse_oracle.c")) as fh:
        source = fh.read()
    assert source.count(_IMAGE) == 1
    # the unmodified source passes both pins
    couette, urel, spread = _pins_with(source, tmp_path, "control")
    assert couette < 1e-7 and urel < 1e-7 and spread < 1e-9
    for name, body in _MUTANTS.items():
        couette, urel, spread = _pins_with(source.replace(_IMAGE, body), tmp_path,
                                           name.replace(" ", "_"))
        assert couette > 1e-3 or urel > 1e-3, (name, couette, urel, spread)
