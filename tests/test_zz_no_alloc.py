"""The entry point that allocates nothing (vanse_observe_noalloc) against
vanse_observe through the C ABI: two calls in a row on one device, the
second on a smaller lattice, each equal to vanse_observe's record."""
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


def _lattice(nx, ny, prec, bc, drag=False, mask=False, rows=None, seed=3):
    from paper_2409_02964_amd.vanse import Lattice
    phi = W.channel_phi(nx, ny, seed=seed)
    lat = Lattice(nx, ny, precision=prec, bc_y=bc, drag=drag, mask=mask)
    lat.set_params(0.5, RATES).set_body_force(2e-5, -1e-5)
    if mask:
        lat.set_mask(W.solid_mask(nx, ny, seed=seed))
    lat.set_void_fraction(phi)
    if drag:
        lat.set_drag(1e-3 + 2e-2 * (1 - phi), (1e-4, 0.0))
    if rows:
        lat.set_velocity_rows(*rows)
    f = W.random_populations(nx, ny, seed=seed + 1)
    lat.set_populations(f).step(7)
    return lat


def test_noalloc_observe_equals_observe_twice():
    _torch()
    cases = [
        (700, 300, "f32s", "wall", dict(drag=True)),                       # 3 x 300 blocks
        (45, 23, "f64", "wall", dict(mask=True)),                          # smaller second call
        (130, 17, "f16s", "wall", dict(rows=(2e-3, None))),
    ]
    for nx, ny, prec, bc, kw in cases:
        _say(f"noalloc observe: {nx}x{ny} {prec} {bc} {kw}")
        lat = _lattice(nx, ny, prec, bc, **kw)
        ref = lat.observe()
        got = lat.observe(noalloc=True)
        _say(f"  observe {ref}\n  noalloc {got}")
        assert got == ref                       # bitwise: same kernels, same order
        assert lat.observe(noalloc=True) == ref  # and again, after another call's data
        lat.close()


def test_noalloc_observe_reports_divergence():
    torch = _torch()
    from paper_2409_02964_amd.vanse import Diverged, Lattice
    lat = Lattice(64, 48, precision="f32s")
    lat.set_params(0.5, RATES).set_void_fraction(np.full((48, 64), 0.8))
    f = W.random_populations(64, 48, seed=2)
    f[5, 10, 11] = np.inf
    lat.set_populations(torch.from_numpy(f)).step(2)
    ref = lat.observe(raise_on_diverged=False)
    got = lat.observe(raise_on_diverged=False, noalloc=True)
    assert got == ref and got["nonfinite"] >= 1
    with pytest.raises(Diverged):
        lat.observe(noalloc=True)
