"""Lattices at the largest size the library accepts (GPU).

A population buffer must stay below 4 GiB (the step kernels address it with
32-bit offsets); at 8192 columns that allows 7281 rows in FP64, 14563 in
FP32 and 29127 in FP16.  The void fraction here repeats in x with period 8,
and so does the state started from a uniform equilibrium: the streaming and
the Eq. (10) stencil see the same neighbours at x and at x + 8.  The largest
lattice must therefore repeat, column for column, a lattice 8 columns wide --
within the FP64 tolerance against the oracle, and bitwise against the GPU's
own 8-column lattice (a node's arithmetic does not depend on its tile).  The
last rows of each plane, where an offset that overflowed would land, are
compared like every other row.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NX, PERIOD = 8192, 8
RATES = dict(s_c=1.2, s_e=1.2, s_eps=1.2, s_q=1.2, s_nu=0.8)
G = (1e-5, 2e-6)
BYTES = {"f64": 8, "f32s": 4, "f16s": 2}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def max_rows(prec):
    return (2 ** 32 - 1) // (9 * BYTES[prec] * NX)


def narrow_phi(ny, seed=7):
    """phi on an 8-column lattice: a wall-to-wall tanh step plus noise"""
    rng = np.random.default_rng(seed)
    y = (np.arange(ny)[:, None] + 0.5) / ny
    return np.clip(0.7 + 0.25 * np.tanh((y - 0.5) * 20) + 0.04 * rng.standard_normal((ny, PERIOD)),
                   0.3, 1.0)


def lattice(nx, ny, prec, phi, spp):
    from paper_2409_02964_amd.vanse import Lattice
    lat = Lattice(nx, ny, precision=prec, bc_y="wall")
    lat.set_params(0.5, RATES).set_body_force(*G).set_void_fraction(phi)
    if spp == 2:
        lat.set_steps_per_pass(2)
        assert lat.fused_tiling()["active"]
    return lat.init_equilibrium(1.0)


def periodic_mismatch(torch, f, fn):
    """max |f[..., x] - fn[..., x mod 8]| over the big lattice, plane by plane"""
    ny = f.shape[1]
    worst = 0.0
    for i in range(9):
        d = f[i].view(ny, NX // PERIOD, PERIOD) - fn[i][:, None, :]
        worst = max(worst, float(d.abs().max()))
    return worst


@pytest.mark.parametrize("spp", [1, 2])
def test_largest_fp64_lattice_against_oracle(oracle, spp):
    torch = _torch()
    ny = max_rows("f64")
    phi = narrow_phi(ny)
    _say(f"FP64 {NX} x {ny} ({9 * NX * ny * 8 / 2**30:.3f} GiB per buffer), "
         f"{spp} step(s) per launch, 3 steps")
    lat = lattice(NX, ny, "f64", np.tile(phi, (1, NX // PERIOD)), spp)
    lat.step(3)
    f = lat.read_populations()
    lat.close()
    o = oracle.Oracle(PERIOD, ny, phi, kappa=0.5, rates=RATES, g=G, bc_y="wall").init_equilibrium()
    o.step(3)
    fo = torch.from_numpy(o.f).to(f.device)
    err = periodic_mismatch(torch, f, fo)
    scale = float(fo.abs().max())
    _say(f"   max |f - f_oracle| = {err:.3e} (max |f| = {scale:.3e})")
    assert err <= 1e-14 * scale


@pytest.mark.parametrize("prec,spp", [("f32s", 1), ("f32s", 2), ("f16s", 2)])
def test_largest_lattice_repeats_narrow_one_bitwise(prec, spp):
    torch = _torch()
    ny = max_rows(prec)
    phi = narrow_phi(ny, seed=8)
    _say(f"{prec} {NX} x {ny} ({9 * NX * ny * BYTES[prec] / 2**30:.3f} GiB per buffer), "
         f"{spp} step(s) per launch, 4 steps")
    small = lattice(PERIOD, ny, prec, phi, spp)
    f0n = small.read_populations()
    fn = small.step(4).read_populations()
    small.close()
    lat = lattice(NX, ny, prec, np.tile(phi, (1, NX // PERIOD)), spp).step(4)
    f = lat.read_populations()
    lat.close()
    assert bool(torch.isfinite(fn).all())
    assert bool((fn[:, -1] != f0n[:, -1]).any())  # the state moved up to the last row
    err = periodic_mismatch(torch, f, fn)
    _say(f"   max |f - f_narrow| = {err:.3e}")
    assert err == 0.0
