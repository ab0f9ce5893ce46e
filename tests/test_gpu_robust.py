"""Race and coverage checks of the step kernels (GPU).

* Every node written: the buffer a launch writes is filled with NaN first;
  after the launch no population may be NaN, so no node of the lattice was
  skipped by the tiling (ragged tails, wall rows, tiny lattices, the second
  step of a two-step launch, members of a batch).
* Determinism: the two-step kernel overlaps its LDS staging with compute
  under hand-placed waits; a missing wait would show as results that differ
  from run to run, so two runs must agree bitwise.
* Independence: lattices and batches stepped concurrently on several
  streams give the results of stepping them one after the other.
* Checkpoint and resume: populations read out and set again continue
  bitwise; a non-finite node is reported as divergence.
"""
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


def lattice(nx, ny, precision, bc, drag=False, seed=3):
    from paper_2409_02964_amd.vanse import Lattice
    phi = W.channel_phi(nx, ny, seed=seed) if ny > 2 else np.full((ny, nx), 0.7)
    lat = Lattice(nx, ny, precision=precision, bc_y=bc, drag=drag)
    lat.set_params(0.5, RATES).set_body_force(2e-5, -1e-5).set_void_fraction(phi)
    if drag:
        lat.set_drag(1e-3 + 2e-2 * (1 - phi), (1e-4, 0.0))
    return lat


def start_state(lat, seed):
    """Rest-state weights perturbed by 2% noise, as FP64 populations."""
    rng = np.random.default_rng(seed)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    return w[:, None, None] * (1.0 + 0.02 * rng.standard_normal((9, lat.ny, lat.nx)))


def nan_destination(lat, f0):
    """Leave NaN in the buffer the next launch writes, then make f0 current.

    A NaN state stepped once by the one-step kernel at its default tiling
    lands, NaN at every node, in the second buffer (that kernel writes every
    node: the FP64 one-step parity tests compare every population with the
    oracle); setting f0 again makes the first buffer current, so the next
    launch reads f0 and writes over the NaN."""
    lat.set_populations(np.full((9, lat.ny, lat.nx), np.nan)).step(1)
    assert np.isnan(lat.read_populations().cpu().numpy()).all()
    lat.set_populations(f0)


SHAPES = [
    (300, 70, "periodic"),
    (253, 130, "wall"),
    (97, 2, "wall"),
    (1000, 37, "wall"),
    (247, 33, "periodic"),
    (246, 20, "wall"),
    (3, 5, "periodic"),
    (2, 2, "periodic"),
]


@pytest.mark.parametrize("nx,ny,bc", SHAPES)
@pytest.mark.parametrize("precision", ["f64", "f32s", "f16s"])
@pytest.mark.parametrize("tiling", [(64, 3), (256, 1), (512, 64)])
def test_one_step_writes_every_node(nx, ny, bc, precision, tiling):
    _torch()
    lat = lattice(nx, ny, precision, bc)
    f0 = start_state(lat, nx + ny)
    nan_destination(lat, f0)
    lat.set_tiling(*tiling).step(1)
    f = lat.read_populations().cpu().numpy()
    _say(f"one step {precision} {nx}x{ny} {bc} tiling {tiling}: {np.isnan(f).sum()} NaN")
    assert np.isfinite(f).all()


@pytest.mark.parametrize("nx,ny,bc", SHAPES)
@pytest.mark.parametrize("precision", ["f64", "f32", "f32s", "f16s"])
@pytest.mark.parametrize("rows", [0, 1, 3])
def test_two_step_writes_every_node(nx, ny, bc, precision, rows):
    _torch()
    lat = lattice(nx, ny, precision, bc)
    f0 = start_state(lat, nx + 2 * ny)
    nan_destination(lat, f0)
    lat.set_steps_per_pass(2, rows)
    if not lat.fused_tiling()["active"]:
        pytest.skip("two-step kernel not taken for this lattice")
    lat.step(2)
    f = lat.read_populations().cpu().numpy()
    _say(f"two steps {precision} {nx}x{ny} {bc} rows {rows}: {np.isnan(f).sum()} NaN")
    assert np.isfinite(f).all()


@pytest.mark.parametrize("spp,precision", [(1, "f64"), (1, "f16s"), (2, "f32s"), (2, "f16s")])
def test_batch_writes_every_node(spp, precision):
    _torch()
    from paper_2409_02964_amd.vanse import Batch
    sizes = [(64, 64, "wall"), (37, 53, "wall"), (130, 20, "wall"), (17, 5, "wall"), (300, 31, "wall")]
    lats = []
    for k, (nx, ny, bc) in enumerate(sizes):
        lat = lattice(nx, ny, precision, bc, seed=k)
        nan_destination(lat, start_state(lat, k))
        lats.append(lat)
    Batch(lats, threads=128, rows=5, steps_per_pass=spp).step(spp)
    for lat in lats:
        f = lat.read_populations().cpu().numpy()
        assert lat.t == spp
        assert np.isfinite(f).all(), f"{lat.nx}x{lat.ny}: {np.isnan(f).sum()} NaN"


@pytest.mark.parametrize("precision,drag", [("f32s", False), ("f16s", False), ("f32s", True),
                                            ("f64", False)])
def test_two_step_determinism(precision, drag):
    """Two runs of 40 steps on a lattice of many tiles agree bitwise."""
    _torch()
    nx, ny = 1500, 700
    res = []
    for _ in range(2):
        lat = lattice(nx, ny, precision, "wall", drag=drag, seed=11)
        lat.set_steps_per_pass(2).init_equilibrium(1.0)
        assert lat.fused_tiling()["active"]
        lat.step(40)
        res.append(lat.read_populations().cpu().numpy())
    assert np.array_equal(res[0], res[1])


def variant_lattice(nx, ny, precision, bc, variant, seed=3):
    """Lattices of the two-step variants beyond the plain step: solid nodes
    (a seeded mask), with the drag, a moving phi with the drag, or model B
    (with the drag)."""
    from paper_2409_02964_amd.vanse import Lattice
    phi = W.channel_phi(nx, ny, seed=seed) if ny > 2 else np.full((ny, nx), 0.7)
    mask = variant.startswith("mask")
    drag = variant.endswith("drag")
    lat = Lattice(nx, ny, precision=precision, bc_y=bc, mask=mask, drag=drag,
                  dynamic_phi=variant.startswith("dyn"))
    lat.set_params(0.5, RATES).set_body_force(2e-5, -1e-5)
    if mask:
        lat.set_mask(W.solid_mask(nx, ny, seed=seed))
    if "model_b" in variant:
        lat.set_scheme("B", 3)
    if "appb" in variant:
        lat.set_scheme("A", 2)
    lat.set_void_fraction(phi)
    if drag:
        lat.set_drag(1e-3 + 2e-2 * (1 - phi), (1e-4, 0.0))
    return lat, phi


@pytest.mark.parametrize("nx,ny,bc", [(300, 70, "periodic"), (253, 130, "wall"), (97, 3, "wall"),
                                      (1000, 37, "wall"), (7, 6, "periodic")])
@pytest.mark.parametrize("precision,variant", [("f32s", "mask"), ("f16s", "mask"), ("f64", "mask"),
                                               ("f32s", "mask_drag"), ("f64", "mask_drag"),
                                               ("f32s", "dyn_drag"), ("f64", "dyn_drag"), ("f16s", "dyn"),
                                               ("f32s", "model_b"), ("f16s", "model_b_drag"), ("f64", "model_b"),
                                               ("f32s", "appb"), ("f16s", "appb_drag"), ("f64", "appb"),
                                               ("f32s", "mask_model_b"), ("f32s", "mask_model_b_drag"),
                                               ("f32s", "mask_appb"), ("f64", "mask_appb_drag")])
def test_two_step_variants_write_every_node(nx, ny, bc, precision, variant):
    """The two-step instances of solid nodes and of a moving phi leave no
    fluid node of the destination unwritten (a moving phi handed over for
    the two steps; solid nodes always read back as the rest state)."""
    _torch()
    lat, phi = variant_lattice(nx, ny, precision, bc, variant, seed=nx + ny)
    f0 = start_state(lat, nx + 3 * ny)
    fluid = np.ones((ny, nx), bool)
    if variant.startswith("mask"):
        fluid = W.solid_mask(nx, ny, seed=nx + ny) == 0
    lat.set_populations(np.full((9, ny, nx), np.nan)).step(1)
    assert np.isnan(lat.read_populations().cpu().numpy()[:, fluid]).all()
    lat.set_populations(f0)
    lat.set_steps_per_pass(2)
    assert lat.fused_tiling()["active"]
    if variant.startswith("dyn"):
        lat.set_void_fraction_next2(np.clip(phi * 0.999, 0.3, 1.0), np.clip(phi * 0.998, 0.3, 1.0))
    lat.step(2)
    f = lat.read_populations().cpu().numpy()
    _say(f"two steps {variant} {precision} {nx}x{ny} {bc}: {np.isnan(f).sum()} NaN")
    assert np.isfinite(f).all()


@pytest.mark.parametrize("precision,variant", [("f32s", "mask"), ("f32s", "mask_drag"), ("f32s", "dyn_drag"),
                                               ("f16s", "mask"), ("f32s", "model_b_drag"), ("f32s", "appb_drag")])
def test_two_step_variant_determinism(precision, variant):
    """Two runs of 40 steps of the solid-node and moving-phi instances on a
    lattice of many tiles agree bitwise."""
    _torch()
    nx, ny = 1500, 700
    res = []
    for _ in range(2):
        lat, phi = variant_lattice(nx, ny, precision, "wall", variant, seed=11)
        lat.set_steps_per_pass(2).init_equilibrium(1.0)
        assert lat.fused_tiling()["active"]
        for k in range(20):
            if variant.startswith("dyn"):
                lat.set_void_fraction_next2(np.clip(phi * (1 - 1e-3 * (2 * k + 1)), 0.3, 1.0),
                                            np.clip(phi * (1 - 1e-3 * (2 * k + 2)), 0.3, 1.0))
            lat.step(2)
        res.append(lat.read_populations().cpu().numpy())
    assert np.array_equal(res[0], res[1])


def test_two_step_batch_determinism():
    _torch()
    from paper_2409_02964_amd.vanse import Batch, Lattice
    specs = W.batch_lattices(24, seed=2)
    res = []
    for _ in range(2):
        lats = []
        for sp in specs:
            lat = Lattice(sp["L"], sp["L"], precision="f16s", bc_y="wall")
            lat.set_params(0.5, RATES).set_body_force(sp["g"], 0.0).set_void_fraction(sp["phi"])
            lat.init_equilibrium(1.0)
            lats.append(lat)
        Batch(lats, threads=128, graph_steps=8, steps_per_pass=2).step(16)
        res.append([l.read_populations().cpu().numpy() for l in lats])
    for a, b in zip(*res):
        assert np.array_equal(a, b)


def test_concurrent_streams_match_sequential():
    """Lattices and a batch stepped at the same time on three streams share
    no device state: every result equals stepping them one after the other."""
    torch = _torch()
    from paper_2409_02964_amd.vanse import Batch

    def make():
        a = lattice(300, 120, "f32s", "wall").set_steps_per_pass(2)
        b = lattice(257, 90, "f16s", "periodic")
        c = [lattice(n, n, "f32", "wall", seed=n) for n in (40, 96, 130)]
        for x in [a, b] + c:
            x.init_equilibrium(1.0)
        return a, b, c

    a0, b0, c0 = make()
    bt0 = Batch(c0, threads=128, steps_per_pass=2)
    for _ in range(10):
        a0.step(3)
        b0.step(3)
        bt0.step(3)
    torch.cuda.synchronize()
    a1, b1, c1 = make()
    bt1 = Batch(c1, threads=128, steps_per_pass=2)
    torch.cuda.synchronize()
    s = [torch.cuda.Stream() for _ in range(3)]
    for _ in range(10):
        a1.step(3, stream=s[0])
        b1.step(3, stream=s[1])
        bt1.step(3, stream=s[2])
    torch.cuda.synchronize()
    for x, y in zip([a0, b0] + c0, [a1, b1] + c1):
        assert x.t == y.t == 30
        assert torch.equal(x.read_populations(), y.read_populations())


@pytest.mark.parametrize("precision,spp", [("f64", 1), ("f64", 2), ("f32", 1), ("f32s", 2),
                                           ("f16s", 1), ("f16s", 2)])
def test_checkpoint_resume_is_bitwise(precision, spp):
    """Populations read out (FP64 f) and set again continue bitwise as if the
    run had never stopped: the stored format decodes to f and encodes back
    exactly (FP64 sums of a stored value and the rest state are exact)."""
    torch = _torch()
    nx, ny = 300, 70
    a = lattice(nx, ny, precision, "wall", drag=True)
    a.set_steps_per_pass(spp).init_equilibrium(1.0, 2e-3, 0.0)
    a.step(7)
    ck = a.read_populations().cpu().numpy()
    a.step(10)
    b = lattice(nx, ny, precision, "wall", drag=True)
    b.set_steps_per_pass(spp).set_populations(ck)
    assert torch.equal(b.read_populations(), torch.from_numpy(ck).to(b.read_populations().device))
    b.step(10)
    assert torch.equal(a.read_populations(), b.read_populations())


def test_non_finite_state_is_reported():
    """A non-finite population is counted by the FP64 observables and raised
    as divergence; it spreads to the node's neighbours with the stream."""
    _torch()
    from paper_2409_02964_amd.vanse import Diverged
    lat = lattice(64, 48, "f32s", "periodic")
    f = start_state(lat, 5)
    f[3, 20, 30] = np.inf
    lat.set_populations(f).step(3)
    o = lat.observe(raise_on_diverged=False)
    assert o["nonfinite"] >= 1
    with pytest.raises(Diverged):
        lat.observe()
    with pytest.raises(Diverged):  # the residual reports it too
        lat.residual()


def test_step_check_interval_reports_divergence():
    """With a check interval the observables run inside vanse_step, and a
    non-finite node (injected as data) makes the call report divergence at
    the first checked time; the steps still run to the end of the call."""
    _torch()
    from paper_2409_02964_amd.vanse import Diverged
    lat = lattice(64, 48, "f32s", "periodic")
    f = start_state(lat, 5)
    f[3, 20, 30] = np.nan
    lat.set_populations(f).set_check_interval(4)
    lat.step(2)                       # no multiple of 4 reached: not checked
    with pytest.raises(Diverged, match="t = 4"):
        lat.step(7)
    assert lat.t == 9


@pytest.mark.parametrize("prec,spp", [("f32s", 1), ("f32s", 2), ("f64", 2)])
def test_step_check_interval_changes_nothing(prec, spp):
    """Checked and unchecked runs of a finite state are bitwise equal, and
    the check's last record is what vanse_observe reports at that time."""
    _torch()
    a = lattice(70, 33, prec, "wall", drag=True)
    b = lattice(70, 33, prec, "wall", drag=True)
    for lat in (a, b):
        lat.set_steps_per_pass(spp).set_populations(start_state(lat, 8))
    a.set_check_interval(3)
    a.step(7).step(5)
    b.step(7).step(5)
    assert a.t == b.t == 12
    assert np.array_equal(a.read_populations().cpu().numpy(), b.read_populations().cpu().numpy())
    assert a.observe() == b.observe()
