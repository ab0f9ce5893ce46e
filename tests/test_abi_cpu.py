"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, sizes workspaces, and validates arguments on the host."""
import ctypes as C
import os
import re

import pytest

from paper_2409_02964_amd import vanse as V

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vanse.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vanse_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = V.lib()
    names = declared_functions()
    assert len(names) >= 19
    for n in names:
        assert hasattr(L, n), n
    assert sorted(V.EXPORTS) == names


def test_library_binds_every_symbol_at_load():
    """Loaded with immediate binding in a fresh process, the library
    resolves every symbol: no launcher is referenced that no translation
    unit instantiates (lazy binding would hide one until it is called)."""
    import subprocess
    import sys
    code = ("import ctypes, os, sys; sys.path.insert(0, %r); from paper_2409_02964_amd import vanse as V; "
            "ctypes.CDLL(V.LIB_PATH, mode=os.RTLD_NOW | os.RTLD_LOCAL)" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]


def test_workspace_bytes_scales_with_precision():
    b64 = V.workspace_bytes(4096, 4096, "f64", "wall")
    b32 = V.workspace_bytes(4096, 4096, "f32", "wall")
    b16 = V.workspace_bytes(4096, 4096, "f16s", "wall")
    plane = 4096 * 4096
    # two population buffers dominate: 2 x 9 planes
    assert b64 >= 18 * plane * 8 and b64 < 18 * plane * 8 + 4 * plane * 8 + (1 << 24)
    assert b32 >= 18 * plane * 4 and b32 < 18 * plane * 4 + 4 * plane * 4 + (1 << 24)
    assert b16 >= 18 * plane * 2 and b16 < b32
    assert V.workspace_bytes(64, 64, "f64", force_field=True) > V.workspace_bytes(64, 64, "f64")


@pytest.mark.parametrize("nx,ny,prec,bcx,bcy,ff,code", [
    (1, 64, 0, 0, 0, 0, -1),
    (64, 1, 0, 0, 0, 0, -1),
    (64, 64, 7, 0, 0, 0, -1),
    (64, 64, 0, 2, 0, 0, -1),
    (64, 64, 0, 0, 5, 0, -1),
    (64, 64, 0, 0, 0, 2, -1),
    (60000, 60000, 1, 0, 0, 0, -1),
    (64, 65536, 3, 0, 0, 0, -1),
])
def test_bad_descriptors_are_rejected(nx, ny, prec, bcx, bcy, ff, code):
    d = V.Desc(nx, ny, prec, bcx, bcy, ff, 0)
    n = C.c_size_t()
    assert V.lib().vanse_workspace_bytes(C.byref(d), C.byref(n)) == code
    assert V.lib().vanse_last_error()


def _fake_handle(nx=64, ny=48, prec=0, bcy=0, mask=0, dynamic=0, bcx=0):
    """A handle over a fake, aligned device address: only host-side calls
    (no HIP work) may be made on it."""
    d = V.Desc(nx, ny, prec, bcx, bcy, 0, 0, mask, dynamic)
    n = C.c_size_t()
    V.check(V.lib().vanse_workspace_bytes(C.byref(d), C.byref(n)))
    h = C.c_void_p()
    assert V.lib().vanse_create(C.byref(d), C.c_void_p(1 << 40), n.value - 1, C.byref(h)) == -2
    assert V.lib().vanse_create(C.byref(d), C.c_void_p((1 << 40) + 8), n.value, C.byref(h)) == -2
    assert V.lib().vanse_create(C.byref(d), None, n.value, C.byref(h)) == -2
    V.check(V.lib().vanse_create(C.byref(d), C.c_void_p(1 << 40), n.value, C.byref(h)))
    return h


def test_host_side_validation():
    L = V.lib()
    h = _fake_handle()
    good = V.Rates(1.0, 1.2, 1.2, 1.4, 1.25)
    assert L.vanse_set_params(h, 0.5, C.byref(good)) == 0
    assert L.vanse_set_params(h, 1.5, C.byref(good)) == -1
    assert L.vanse_set_params(h, -0.1, C.byref(good)) == -1
    for k in range(5):
        vals = [1.0, 1.2, 1.2, 1.4, 1.25]
        vals[k] = 2.0
        assert L.vanse_set_params(h, 0.5, C.byref(V.Rates(*vals))) == -1
        vals[k] = 0.0
        assert L.vanse_set_params(h, 0.5, C.byref(V.Rates(*vals))) == -1
    assert L.vanse_set_body_force(h, 1e-6, 0.0, 1) == 0
    assert L.vanse_set_body_force(h, float("nan"), 0.0, 1) == -1
    assert L.vanse_set_body_force(h, 1e-6, 0.0, 3) == -1
    # stepping or reading before phi and populations: state errors, no GPU work
    assert L.vanse_step(h, 1, None) == -4
    assert L.vanse_read_populations(h, C.c_void_p(1 << 40), None) == -4
    assert L.vanse_init_equilibrium(h, 1.0, 0.0, 0.0, None) == -4
    assert L.vanse_time(h) == 0
    assert L.vanse_set_force_field(h, C.c_void_p(1 << 40), C.c_void_p(1 << 40), None) == -4
    assert L.vanse_set_storage_exponent(h, 40) == -1
    assert L.vanse_set_storage_exponent(h, 10) == 0
    assert L.vanse_destroy(h) == 0


def test_tiling_choices():
    L = V.lib()
    h = _fake_handle(4096, 4096, 1, 1)
    t, r, w = C.c_int(), C.c_int(), C.c_int()
    V.check(L.vanse_get_tiling(h, C.byref(t), C.byref(r), C.byref(w)))
    assert t.value in (64, 128, 256, 512) and r.value >= 1
    strips = -(-4096 // (t.value - 4))
    assert w.value == strips * -(-4096 // r.value)
    assert L.vanse_set_tiling(h, 96, 8) == -1
    assert L.vanse_set_tiling(h, 128, 0) == 0  # back to the default
    assert L.vanse_set_tiling(h, 512, 3) == 0
    V.check(L.vanse_get_tiling(h, C.byref(t), C.byref(r), C.byref(w)))
    assert (t.value, r.value, w.value) == (512, 3, 9 * 1366)
    assert L.vanse_destroy(h) == 0


def test_error_strings():
    L = V.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.vanse_error_string(code)


@pytest.mark.parametrize("mask,dynamic", [(2, 0), (0, 3), (-1, 0)])
def test_bad_feature_flags_are_rejected(mask, dynamic):
    d = V.Desc(64, 64, 0, 0, 0, 0, 0, mask, dynamic)
    n = C.c_size_t()
    assert V.lib().vanse_workspace_bytes(C.byref(d), C.byref(n)) == -1


def test_optional_planes_enlarge_the_workspace():
    base = V.workspace_bytes(100, 80, "f32")
    plane = 128 * 80
    assert V.workspace_bytes(100, 80, "f32", mask=True) >= base + 2 * plane
    assert V.workspace_bytes(100, 80, "f32", dynamic_phi=True) >= base + 4 * plane
    assert V.workspace_bytes(100, 80, "f64", dynamic_phi=True) >= V.workspace_bytes(100, 80, "f64") + 8 * plane


def test_feature_state_checks_on_the_host():
    L = V.lib()
    h = _fake_handle(mask=1, dynamic=1)
    # phi(t+1) needs phi first; stepping needs the mask; both without GPU work
    assert L.vanse_set_void_fraction_next(h, C.c_void_p(1 << 40), None) == -4
    assert L.vanse_set_mask(h, None, None) == -1
    assert L.vanse_step(h, 1, None) == -4
    plain = _fake_handle()
    assert L.vanse_set_mask(plain, C.c_void_p(1 << 40), None) == -4
    assert L.vanse_set_void_fraction_next(plain, C.c_void_p(1 << 40), None) == -4
    assert L.vanse_destroy(h) == 0 and L.vanse_destroy(plain) == 0


def test_two_step_void_fraction_checks_on_the_host():
    """vanse_set_void_fraction_next2 rejects, before any GPU work: a lattice
    without dynamic_phi (-4), a missing phi (-1), a void fraction not set yet
    (-4)."""
    L = V.lib()
    p = C.c_void_p(1 << 40)
    plain = _fake_handle()
    assert L.vanse_set_void_fraction_next2(plain, p, p, None, None, None, None) == -4
    dyn = _fake_handle(dynamic=1)
    assert L.vanse_set_void_fraction_next2(dyn, p, None, None, None, None, None) == -1
    assert L.vanse_set_void_fraction_next2(dyn, None, p, None, None, None, None) == -1
    assert L.vanse_set_void_fraction_next2(dyn, p, p, None, None, None, None) == -4
    assert L.vanse_destroy(plain) == 0 and L.vanse_destroy(dyn) == 0


@pytest.mark.parametrize("first,second,code", [
    (dict(), dict(mask=1), -1),               # members differ in their variant
    (dict(), dict(dynamic=1), -6),            # a moving phi is not batched
    (dict(dynamic=1), dict(dynamic=1), -6),
    (dict(mask=1), dict(mask=1), 0),          # solid nodes are
    (dict(bcx=1), dict(bcx=1, mask=1), 0),    # walls in x, with or without solid nodes
    (dict(bcx=1), dict(mask=1), -1)])         # the same instance, other x boundaries
def test_batch_variant_rules(first, second, code):
    L = V.lib()
    hs = [_fake_handle(**first), _fake_handle(**second)]
    arr = (C.c_void_p * 2)(hs[0].value, hs[1].value)
    n = C.c_size_t()
    assert L.vanse_batch_workspace_bytes(arr, 2, 128, 0, C.byref(n)) == code
    for h in hs:
        assert L.vanse_destroy(h) == 0


def test_scheme_validation_on_the_host():
    L = V.lib()
    h = _fake_handle()
    assert L.vanse_set_scheme(h, 2, 3) == -1
    assert L.vanse_set_scheme(h, 0, 1) == -1
    assert L.vanse_set_scheme(h, 1, 2) == 0
    other = _fake_handle()
    arr = (C.c_void_p * 2)(other.value, h.value)
    n = C.c_size_t()
    assert L.vanse_batch_workspace_bytes(arr, 2, 128, 0, C.byref(n)) == -1  # members differ
    assert L.vanse_set_scheme(other, 1, 2) == 0
    assert L.vanse_batch_workspace_bytes(arr, 2, 128, 0, C.byref(n)) == 0   # same variant
    assert L.vanse_set_scheme(h, 0, 3) == 0
    assert L.vanse_batch_workspace_bytes(arr, 2, 128, 0, C.byref(n)) == -1
    assert L.vanse_set_scheme(other, 0, 3) == 0
    assert L.vanse_batch_workspace_bytes(arr, 2, 128, 0, C.byref(n)) == 0
    assert L.vanse_destroy(h) == 0 and L.vanse_destroy(other) == 0


@pytest.mark.parametrize("prec,sb", [("f64", 8), ("f32", 4), ("f32s", 4), ("f16s", 2)])
def test_largest_lattice_boundary(prec, sb):
    """A population buffer (nine planes) must stay below 4 GiB, since the step
    kernels address it with 32-bit offsets: at 8192 columns the tallest
    lattice below the limit is accepted and one row more is rejected."""
    nx = 8192
    ny = (2 ** 32 - 1) // (9 * sb * nx)
    assert V.workspace_bytes(nx, ny, prec, "wall") > 2 * 9 * sb * nx * ny
    with pytest.raises(V.VanseError, match="too large"):
        V.workspace_bytes(nx, ny + 1, prec, "wall")


def test_tallest_lattice():
    """Rows map to the grid's y dimension of the set-up and read-out kernels."""
    assert V.workspace_bytes(64, 65535, "f16s", "wall") > 0
    with pytest.raises(V.VanseError, match="too tall"):
        V.workspace_bytes(64, 65536, "f16s", "wall")


def test_velocity_rows_validation_on_the_host():
    L = V.lib()
    per = _fake_handle()
    assert L.vanse_set_velocity_rows(per, 2, 0.0, 1e-3) == -4        # no walls
    box = _fake_handle(bcy=1, bcx=1)
    assert L.vanse_set_velocity_rows(box, 2, 0.0, 1e-3) == -6        # walls in x
    solid = _fake_handle(bcy=1, mask=1)
    assert L.vanse_set_velocity_rows(solid, 2, 0.0, 1e-3) == -6      # solid nodes
    thin = _fake_handle(ny=2, bcy=1)
    assert L.vanse_set_velocity_rows(thin, 1, 1e-3, 0.0) == -1       # no fluid row
    h = _fake_handle(bcy=1)
    assert L.vanse_set_velocity_rows(h, 4, 0.0, 1e-3) == -1          # unknown face bit
    assert L.vanse_set_velocity_rows(h, 2, 0.0, float("inf")) == -1
    assert L.vanse_set_wall_velocity(h, 1e-3, 0.0) == 0
    assert L.vanse_set_velocity_rows(h, 1, 1e-3, 0.0) == -1          # the half-way wall moves
    assert L.vanse_set_velocity_rows(h, 2, 0.0, 1e-3) == 0
    assert L.vanse_set_wall_velocity(h, 1e-3, 2e-3) == -1            # face is a velocity row
    other = _fake_handle(bcy=1)
    arr = (C.c_void_p * 2)(h.value, other.value)
    n = C.c_size_t()
    assert L.vanse_batch_workspace_bytes(arr, 1, 128, 0, C.byref(n)) == -6   # not batched
    for x in (per, box, solid, thin, h, other):
        assert L.vanse_destroy(x) == 0


def test_check_interval_validation_on_the_host():
    L = V.lib()
    h = _fake_handle()
    assert L.vanse_set_check_interval(h, -1) == -1
    assert L.vanse_set_check_interval(h, 0) == 0
    assert L.vanse_set_check_interval(h, 100) == 0
    assert L.vanse_step(h, 10, None) == -4                          # still no state: no GPU work
    assert L.vanse_destroy(h) == 0


def test_noalloc_observe_limit_on_the_host():
    """vanse_observe_noalloc keeps its partials in a static array of 131072
    records (one per 256-column block of a row): a larger lattice is refused
    before any device work."""
    L = V.lib()
    big = _fake_handle(nx=513, ny=43691)       # 3 blocks per row: 131073 records
    out = (C.c_double * 4)()
    assert L.vanse_observe_noalloc(big, out, None) == -1
    assert "static scratch" in L.vanse_last_error().decode()
    fits = _fake_handle(nx=512, ny=65535)      # 2 blocks per row: 131070 records
    assert L.vanse_observe_noalloc(fits, out, None) == -4   # fits; no state yet
    assert L.vanse_observe_noalloc(fits, None, None) == -1
    for h in (big, fits):
        assert L.vanse_destroy(h) == 0


def test_two_step_routing_on_the_host():
    """Which lattices take two steps per launch when asked (a host-side
    choice): the plain step and the scheme variants (also with solid nodes)
    do; wall velocities and walls in x keep one.
    Batches with two steps per launch follow the same rule, and their members
    must share the two-step instance."""
    L = V.lib()

    def active(h):
        a, r, w = C.c_int(), C.c_int(), C.c_int()
        V.check(L.vanse_get_fused_tiling(h, C.byref(a), C.byref(r), C.byref(w)))
        return a.value

    def lattice(scheme=None, wall_u=None, **kw):
        h = _fake_handle(**kw)
        if scheme is not None:
            assert L.vanse_set_scheme(h, *scheme) == 0
        if wall_u is not None:
            assert L.vanse_set_wall_velocity(h, 0.0, wall_u) == 0
        assert L.vanse_set_steps_per_pass(h, 2, 0) == 0
        return h

    cases = [(dict(bcy=1), 1), (dict(bcy=1, scheme=(1, 3)), 1), (dict(scheme=(1, 3)), 1),
             (dict(bcy=1, scheme=(1, 2)), 1), (dict(bcy=1, scheme=(0, 2)), 1),
             (dict(bcy=1, scheme=(1, 3), wall_u=1e-3), 0), (dict(bcx=1), 0),
             (dict(bcy=1, mask=1, scheme=(1, 3)), 1), (dict(bcy=1, mask=1, scheme=(0, 2)), 1),
             (dict(bcy=1, mask=1, scheme=(1, 3), wall_u=1e-3), 0),
             (dict(bcy=1, mask=1), 1)]
    for kw, want in cases:
        h = lattice(**kw)
        assert active(h) == want, kw
        assert L.vanse_destroy(h) == 0
    n = C.c_size_t()
    for schemes, code in ((((1, 3), (1, 3)), 0), (((0, 2), (0, 2)), 0), (((1, 3), (0, 2)), -1),
                          (((1, 2), (1, 3)), -1)):
        hs = [lattice(bcy=1, scheme=sc) for sc in schemes]
        arr = (C.c_void_p * 2)(hs[0].value, hs[1].value)
        # (FP64 handles: the Appendix B instance takes halves of at most 64 lanes)
        assert L.vanse_batch_workspace_bytes_ex(arr, 2, 64, 0, 2, C.byref(n)) == code, schemes
        assert L.vanse_batch_workspace_bytes_ex(arr, 2, 64, 0, 1, C.byref(n)) == 0  # one step: alike
        for h in hs:
            assert L.vanse_destroy(h) == 0
