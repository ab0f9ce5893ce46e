// vanse.hip -- libvanse: host side of the C ABI declared in include/vanse.h.
//
// The handle validates arguments, carves all device state out of the
// caller's workspace, picks the template instance of the fused step kernel
// (precision x boundary x force field x workgroup width) and enqueues work on
// the caller's stream.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <type_traits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "aux_kernels.hpp"
#include "step_kernel.hpp"
#include "step_launch.hpp"
#include "vanse.h"

using namespace vanse_dev;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(VANSE_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));   \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

int storage_bytes(int precision) {
  switch (precision) {
    case VANSE_F64: return 8;
    case VANSE_F32: return 4;
    case VANSE_F32_SHIFTED: return 4;
    case VANSE_F16_SHIFTED: return 2;
    default: return 0;
  }
}
int compute_bytes(int precision) { return precision == VANSE_F64 ? 8 : 4; }

int pitch_of(int nx) { return (nx + 63) / 64 * 64; }

struct Layout {
  size_t pop[2], phi, phin, nbr, fx, fy, beta, drho, uprev, partials, partials2, result, badcount,
      check, total;
  // a moving phi: phi(t+2) and the second step's force field and drag
  // coefficient of a two-step hand-over (vanse_set_void_fraction_next2)
  size_t phin2, fx2, fy2, beta2;
  long long plane;
  int pitch;
  long long max_partials;
};

int make_layout(const vanse_desc* d, Layout* L) {
  if (!d) return fail(VANSE_ERR_INVALID_ARG, "desc is NULL");
  if (d->nx < 2 || d->ny < 2) return fail(VANSE_ERR_INVALID_ARG, "nx, ny must be >= 2 (got %d, %d)", d->nx, d->ny);
  // the set-up and read-out kernels launch one grid row per lattice row
  if (d->ny > 65535) return fail(VANSE_ERR_INVALID_ARG, "lattice too tall: ny must be <= 65535 (got %d)", d->ny);
  if (storage_bytes(d->precision) == 0) return fail(VANSE_ERR_INVALID_ARG, "unknown precision %d", d->precision);
  if (d->bc_x != VANSE_PERIODIC && d->bc_x != VANSE_WALL) return fail(VANSE_ERR_INVALID_ARG, "unknown bc_x %d", d->bc_x);
  if (d->bc_y != VANSE_PERIODIC && d->bc_y != VANSE_WALL) return fail(VANSE_ERR_INVALID_ARG, "unknown bc_y %d", d->bc_y);
  if (d->has_force_field != 0 && d->has_force_field != 1) return fail(VANSE_ERR_INVALID_ARG, "has_force_field must be 0 or 1");
  if (d->has_drag != 0 && d->has_drag != 1) return fail(VANSE_ERR_INVALID_ARG, "has_drag must be 0 or 1");
  if (d->has_mask != 0 && d->has_mask != 1) return fail(VANSE_ERR_INVALID_ARG, "has_mask must be 0 or 1");
  if (d->dynamic_phi != 0 && d->dynamic_phi != 1) return fail(VANSE_ERR_INVALID_ARG, "dynamic_phi must be 0 or 1");
  const long long pitch = pitch_of(d->nx);
  const long long plane = pitch * d->ny;
  if (plane * 9 > (1LL << 31) - 1) return fail(VANSE_ERR_INVALID_ARG, "lattice too large (%d x %d)", d->nx, d->ny);
  const size_t sb = storage_bytes(d->precision), cb = compute_bytes(d->precision);
  // the step kernel addresses each population buffer with 32-bit offsets
  if ((unsigned long long)plane * 9ULL * sb >= (1ULL << 32))
    return fail(VANSE_ERR_INVALID_ARG, "lattice too large: one population buffer must stay below 4 GiB "
                "(%d x %d at %zu bytes per population)", d->nx, d->ny, sb);
  size_t off = 0;
  L->pitch = (int)pitch;
  L->plane = plane;
  for (int b = 0; b < 2; ++b) { L->pop[b] = off; off = align256(off + 9 * plane * sb); }
  L->phi = off; off = align256(off + plane * cb);
  L->phin = L->phin2 = L->fx2 = L->fy2 = L->beta2 = 0;
  if (d->dynamic_phi) {
    L->phin = off; off = align256(off + plane * cb);
    L->phin2 = off; off = align256(off + plane * cb);
    if (d->has_force_field) {
      L->fx2 = off; off = align256(off + plane * cb);
      L->fy2 = off; off = align256(off + plane * cb);
    }
    if (d->has_drag) { L->beta2 = off; off = align256(off + plane * cb); }
  }
  L->nbr = 0;
  if (d->has_mask) { L->nbr = off; off = align256(off + plane * sizeof(uint16_t)); }
  if (d->has_force_field) {
    L->fx = off; off = align256(off + plane * cb);
    L->fy = off; off = align256(off + plane * cb);
  } else {
    L->fx = L->fy = 0;
  }
  L->beta = 0;
  if (d->has_drag) { L->beta = off; off = align256(off + plane * cb); }
  L->drho = off; off = align256(off + plane * cb);
  L->uprev = off; off = align256(off + 2 * plane * cb);
  L->max_partials = (long long)((d->nx + 255) / 256) * d->ny;
  L->partials = off; off = align256(off + L->max_partials * NOBS * sizeof(double));
  L->partials2 = off; off = align256(off + 1024 * NOBS * sizeof(double));
  L->result = off; off = align256(off + NOBS * sizeof(double));
  L->badcount = off; off = align256(off + sizeof(unsigned long long));
  L->check = off; off = align256(off + sizeof(long long));
  L->total = off;
  return VANSE_OK;
}

}  // namespace

struct vanse_lattice {
  vanse_desc d;
  Layout L;
  char* ws;
  int cur;  // buffer holding the current state
  int64_t t;
  bool phi_set, params_set, state_set, ff_set, drag_set, uprev_valid, mask_set, phin_set;
  // two steps' void fractions pending (phi(t+1) in L.phin, phi(t+2) in
  // L.phin2), and whether the second step brings its own force field
  // (L.fx2, L.fy2) and drag coefficient (L.beta2)
  bool phin2_set = false, f2_set = false, beta2_set = false;
  double usx, usy;  // solid velocity of the linear drag
  double kappa, rho0, gx, gy;
  int scale_by_phi;
  int model_b, eq2;  // scheme variants (vanse_set_scheme)
  double uw_lo, uw_hi;  // wall velocities (vanse_set_wall_velocity)
  int nee_lo, nee_hi;   // velocity boundary rows (vanse_set_velocity_rows)
  double un_lo, un_hi;
  vanse_rates rates;
  int threads, rows;  // launch shape of the step kernel
  int fuse;           // time steps per launch of the plain step (1 or 2)
  int rows2;          // rows per workgroup of the two-step kernel (0: default)
  bool tiling_default;
  int storage_exp;
  long long version;  // bumped by every call that changes what the step reads
  int64_t check_every;  // vanse_step runs the observables at multiples of this t (0: never)
};

namespace {

// Compute units of the current device (256 on MI355X when no device is
// visible, so that host-only use of the ABI still gets a tiling).
int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
    return cus;
  (void)hipGetLastError();
  return 256;
}

// Default launch shape: 256-lane workgroups on wide lattices, and rows per
// workgroup chosen so that the grid is one full round of resident
// workgroups (4 per CU for the FP32 kernels, 2 for FP64): every workgroup
// then sweeps the same number of rows and none waits in a second round.  A
// lattice too small to fill that round gets fewer rows per workgroup, down
// to one: it is bound by the sweep's latency (about a microsecond per row),
// not by the extra halo rows (measured: 64^2 FP64 5.6 us per step with one
// row, 9.2 with four).
void default_tiling(vanse_lattice* h) {
  const int nx = h->d.nx, ny = h->d.ny;
  const int threads = nx >= 200 ? 256 : (nx >= 100 ? 128 : 64);
  const int strips = (nx + threads - 5) / (threads - 4);
  const int per_cu = (h->d.precision == VANSE_F64 ? 2 : 4) * (256 / threads);
  const long long slots = (long long)device_cus() * per_cu;
  long long nby = slots / strips;
  if (nby < 1) nby = 1;
  const long long r = (ny + nby - 1) / nby;
  h->threads = threads;
  h->rows = (int)r;
}

template <typename T>
StepPhys<T> make_phys(const vanse_lattice* h) {
  StepPhys<T> p;
  p.kappa = T(h->kappa);
  p.rho0 = T(h->rho0);
  p.gx = T(h->gx);
  p.gy = T(h->gy);
  p.s_e = T(h->rates.s_e);
  p.s_eps = T(h->rates.s_eps);
  p.s_q = T(h->rates.s_q);
  p.s_nu = T(h->rates.s_nu);
  p.rest_axis = T(h->kappa * h->rho0 / 9.0);
  p.rest_diag = T(h->kappa * h->rho0 / 36.0);
  p.rest0_k = T(5.0 * h->kappa * h->rho0 / 9.0);
  const bool half = h->d.precision == VANSE_F16_SHIFTED;
  p.scale = T(half ? std::ldexp(1.0, h->storage_exp) : 1.0);
  p.inv_scale = T(half ? std::ldexp(1.0, -h->storage_exp) : 1.0);
  p.usx = T(h->usx);
  p.usy = T(h->usy);
  p.scale_by_phi = h->scale_by_phi;
  p.model_b = h->model_b;
  p.eq2 = h->eq2;
  p.uw_lo = T(h->uw_lo);
  p.uw_hi = T(h->uw_hi);
  p.k2 = T(2) * p.kappa;
  p.k3 = T(3) * p.kappa;
  p.k12 = p.kappa * T(1.0 / 12.0);
  p.he = T(1) - T(0.5) * p.s_e;
  p.hep = T(1) - T(0.5) * p.s_eps;
  p.hq = T(1) - T(0.5) * p.s_q;
  p.hn = T(1) - T(0.5) * p.s_nu;
  p.bt9 = p.scale * T(1.0 / 9.0);
  p.bt36 = p.scale * T(1.0 / 36.0);
  p.bt6 = p.scale * T(1.0 / 6.0);
  p.bt12 = p.scale * T(1.0 / 12.0);
  p.bt4 = p.scale * T(0.25);
  p.nee_lo = h->nee_lo;
  p.nee_hi = h->nee_hi;
  p.un_lo = T(h->un_lo);
  p.un_hi = T(h->un_hi);
  return p;
}

Geo make_geo(const vanse_lattice* h) {
  Geo G;
  G.nx = h->d.nx;
  G.ny = h->d.ny;
  G.pitch = h->L.pitch;
  G.walls = h->d.bc_y == VANSE_WALL;
  G.xwalls = h->d.bc_x == VANSE_WALL;
  G.plane = h->L.plane;
  G.nee_lo = h->nee_lo;
  G.nee_hi = h->nee_hi;
  G.un_lo = h->un_lo;
  G.un_hi = h->un_hi;
  return G;
}

template <typename S, typename T, bool SHIFT, bool WALLS, int FEAT>
int launch_step_w(const vanse_lattice* h, const StepGeom& g, const StepPhys<T>& ph, int blocks,
                  hipStream_t st) {
  switch (h->threads) {
    case 64: launch_step_nt<S, T, SHIFT, WALLS, FEAT, 64>(g, ph, blocks, st); break;
    case 128: launch_step_nt<S, T, SHIFT, WALLS, FEAT, 128>(g, ph, blocks, st); break;
    case 256: launch_step_nt<S, T, SHIFT, WALLS, FEAT, 256>(g, ph, blocks, st); break;
    case 512:
      if constexpr (FEAT == 0) {
        launch_step_nt<S, T, SHIFT, WALLS, FEAT, 512>(g, ph, blocks, st);
        break;
      }
      return fail(VANSE_ERR_UNSUPPORTED, "512-lane workgroups are built for the plain step only");
    default: return fail(VANSE_ERR_INVALID_ARG, "unsupported workgroup width %d", h->threads);
  }
  return VANSE_OK;
}

// Specialised step variants: the force field and the drag; a time-varying
// void fraction with either or both (one instance, FEAT_MOVING, whose absent
// planes read as zero); solid nodes alone (FEAT_MASK), with the force field
// or the drag (FEAT_MASK | FEAT_FORCE | FEAT_DRAG) or with a moving phi
// (FEAT_MASK | FEAT_MOVING); the scheme variants with any of those
// (FEAT_SCHEME | FEAT_MOVING).  Scheme variants with solid nodes use
// FEAT_ALL.  Walls in x take the solid-node instances, with or without a
// mask (an absent flag plane reads as zero); with a force field or drag the
// moving-phi one (FEAT_MASK | FEAT_FORCE | FEAT_DRAG is built without them).
constexpr int FEAT_MOVING = FEAT_DYNPHI | FEAT_FORCE | FEAT_DRAG;
int feat_of(const vanse_lattice* h) {
  const vanse_desc& d = h->d;
  const bool scheme = h->model_b || h->eq2 || h->uw_lo != 0.0 || h->uw_hi != 0.0;
  if (h->nee_lo || h->nee_hi) return FEAT_ALL;  // velocity rows: built there only
  if (d.has_mask || d.bc_x == VANSE_WALL) {
    if (scheme) return FEAT_ALL;
    if (d.dynamic_phi || (d.bc_x == VANSE_WALL && (d.has_force_field || d.has_drag)))
      return FEAT_MASK | FEAT_MOVING;
    return (d.has_force_field || d.has_drag) ? (FEAT_MASK | FEAT_FORCE | FEAT_DRAG) : FEAT_MASK;
  }
  if (scheme) return FEAT_SCHEME | FEAT_MOVING;
  if (d.dynamic_phi) return FEAT_MOVING;
  return (d.has_force_field ? FEAT_FORCE : 0) | (d.has_drag ? FEAT_DRAG : 0);
}

// Lattices batches take: any variant with an instance of its own (not
// FEAT_ALL) and no moving phi (its phi(t+1) is given step by step)
bool batch_ok(const vanse_lattice* h) { return !h->d.dynamic_phi && feat_of(h) != FEAT_ALL; }

// Call fn(std::integral_constant<bool, WALLS>, std::integral_constant<int, FEAT>).
template <typename Fn>
int by_variant(const vanse_lattice* h, Fn&& fn) {
  const bool walls = h->d.bc_y == VANSE_WALL;
  switch (feat_of(h)) {
    case FEAT_ALL: return walls ? fn(std::true_type{}, std::integral_constant<int, FEAT_ALL>{}) : fn(std::false_type{}, std::integral_constant<int, FEAT_ALL>{});
    case FEAT_SCHEME | FEAT_MOVING: return walls ? fn(std::true_type{}, std::integral_constant<int, FEAT_SCHEME | FEAT_MOVING>{}) : fn(std::false_type{}, std::integral_constant<int, FEAT_SCHEME | FEAT_MOVING>{});
    case FEAT_MASK | FEAT_MOVING: return walls ? fn(std::true_type{}, std::integral_constant<int, FEAT_MASK | FEAT_MOVING>{}) : fn(std::false_type{}, std::integral_constant<int, FEAT_MASK | FEAT_MOVING>{});
    case FEAT_MASK | FEAT_FORCE | FEAT_DRAG: return walls ? fn(std::true_type{}, std::integral_constant<int, FEAT_MASK | FEAT_FORCE | FEAT_DRAG>{}) : fn(std::false_type{}, std::integral_constant<int, FEAT_MASK | FEAT_FORCE | FEAT_DRAG>{});
    case FEAT_MASK: return walls ? fn(std::true_type{}, std::integral_constant<int, FEAT_MASK>{}) : fn(std::false_type{}, std::integral_constant<int, FEAT_MASK>{});
    case FEAT_MOVING: return walls ? fn(std::true_type{}, std::integral_constant<int, FEAT_MOVING>{}) : fn(std::false_type{}, std::integral_constant<int, FEAT_MOVING>{});
    case 0: return walls ? fn(std::true_type{}, std::integral_constant<int, 0>{}) : fn(std::false_type{}, std::integral_constant<int, 0>{});
    case 1: return walls ? fn(std::true_type{}, std::integral_constant<int, 1>{}) : fn(std::false_type{}, std::integral_constant<int, 1>{});
    case 2: return walls ? fn(std::true_type{}, std::integral_constant<int, 2>{}) : fn(std::false_type{}, std::integral_constant<int, 2>{});
    default: return walls ? fn(std::true_type{}, std::integral_constant<int, 3>{}) : fn(std::false_type{}, std::integral_constant<int, 3>{});
  }
}

// Two-step launches of the plain step with any of the force field, the
// linear drag and solid nodes (no walls in x, moving phi or scheme variant).
// Halves of step2_nt_of lanes (256 in FP32 arithmetic and 128 in FP64, fewer
// with solid nodes); each outputs its half's width less 10 columns.  Rows per
// workgroup default to one full round of resident workgroups.
int arith_bytes(const vanse_lattice* h) { return h->d.precision == VANSE_F64 ? 8 : 4; }
// The two-step instance of a lattice, or -1 for a variant the two-step
// kernel does not take (walls in x, the Appendix B equilibrium, wall
// velocities, velocity rows, solid nodes with a moving phi or a scheme
// variant): its single-step variant, except that solid nodes without a force
// field take an instance without the force planes (FEAT_MASK, or FEAT_MASK |
// FEAT_DRAG with the drag; the per-row loads of the force field into
// registers make the sweep wait for the rows staged ahead as well), a moving
// phi takes FEAT_DYNPHI with the drag and the force field it has, model B
// alone takes FEAT_SCHEME, with FEAT_DRAG for the drag alone and FEAT_FORCE
// | FEAT_DRAG with the force field, and the Appendix B equilibrium (with or
// without model B) FEAT_EQ2, with FEAT_FORCE | FEAT_DRAG when it has either.
// The scheme variants with solid nodes (FEAT_ALL in one step per launch)
// take FEAT_MASK with FEAT_EQ2 (the Appendix B equilibrium, with or without
// model B) or FEAT_SCHEME (model B alone), with FEAT_FORCE | FEAT_DRAG when
// they have either.
int fused_inst(const vanse_lattice* h) {
  const int f = feat_of(h);
  if (h->d.bc_x == VANSE_WALL) return -1;
  if (f == FEAT_ALL) {
    if (!h->d.has_mask || !(h->model_b || h->eq2) || h->uw_lo != 0.0 || h->uw_hi != 0.0 || h->nee_lo ||
        h->nee_hi || h->d.dynamic_phi)
      return -1;
    const int fd = (h->d.has_force_field || h->d.has_drag) ? (FEAT_FORCE | FEAT_DRAG) : 0;
    return FEAT_MASK | (h->eq2 ? FEAT_EQ2 : FEAT_SCHEME) | fd;
  }
  if (f == (FEAT_SCHEME | FEAT_MOVING)) {
    if (h->uw_lo != 0.0 || h->uw_hi != 0.0 || h->d.dynamic_phi) return -1;
    const bool fd = h->d.has_force_field || h->d.has_drag;
    if (h->eq2) return fd ? (FEAT_EQ2 | FEAT_FORCE | FEAT_DRAG) : FEAT_EQ2;
    if (!h->model_b) return -1;
    if (h->d.has_force_field) return FEAT_SCHEME | FEAT_FORCE | FEAT_DRAG;
    return h->d.has_drag ? (FEAT_SCHEME | FEAT_DRAG) : FEAT_SCHEME;
  }
  if (h->d.dynamic_phi) {
    if (f != FEAT_MOVING) return -1;
    return FEAT_DYNPHI | (h->d.has_force_field ? (FEAT_FORCE | FEAT_DRAG) : (h->d.has_drag ? FEAT_DRAG : 0));
  }
  if ((f & ~(FEAT_FORCE | FEAT_DRAG | FEAT_MASK)) != 0) return -1;
  if ((f & FEAT_MASK) && !h->d.has_force_field) return h->d.has_drag ? (FEAT_MASK | FEAT_DRAG) : FEAT_MASK;
  return f;
}
int fused_nt_of(const vanse_lattice* h) { return step2_nt_of(arith_bytes(h), std::max(fused_inst(h), 0)); }
int fused_out_w(const vanse_lattice* h) { return fused_nt_of(h) - 10; }

bool fused_feat(const vanse_lattice* h) { return fused_inst(h) >= 0; }

bool fused_ok(const vanse_lattice* h) { return h->fuse == 2 && fused_feat(h); }

// LDS bytes of a two-step workgroup of the variant feat
template <typename S, typename T>
unsigned fused_lds_bytes(int feat) {
  auto of = [](auto f) {
    constexpr int F = decltype(f)::value;
    return step2_lds_bytes<S, T, F, step2_nt_of(int(sizeof(T)), F)>();
  };
  switch (feat) {
    case FEAT_DRAG: return of(std::integral_constant<int, FEAT_DRAG>{});
    case FEAT_FORCE: return of(std::integral_constant<int, FEAT_FORCE>{});
    case FEAT_FORCE | FEAT_DRAG: return of(std::integral_constant<int, FEAT_FORCE | FEAT_DRAG>{});
    case FEAT_MASK: return of(std::integral_constant<int, FEAT_MASK>{});
    case FEAT_MASK | FEAT_DRAG: return of(std::integral_constant<int, FEAT_MASK | FEAT_DRAG>{});
    case FEAT_MASK | FEAT_FORCE | FEAT_DRAG:
      return of(std::integral_constant<int, FEAT_MASK | FEAT_FORCE | FEAT_DRAG>{});
    case FEAT_DYNPHI: return of(std::integral_constant<int, FEAT_DYNPHI>{});
    case FEAT_DYNPHI | FEAT_DRAG: return of(std::integral_constant<int, FEAT_DYNPHI | FEAT_DRAG>{});
    case FEAT_DYNPHI | FEAT_FORCE | FEAT_DRAG:
      return of(std::integral_constant<int, FEAT_DYNPHI | FEAT_FORCE | FEAT_DRAG>{});
    case FEAT_SCHEME: return of(std::integral_constant<int, FEAT_SCHEME>{});
    case FEAT_SCHEME | FEAT_DRAG: return of(std::integral_constant<int, FEAT_SCHEME | FEAT_DRAG>{});
    case FEAT_SCHEME | FEAT_FORCE | FEAT_DRAG:
      return of(std::integral_constant<int, FEAT_SCHEME | FEAT_FORCE | FEAT_DRAG>{});
    case FEAT_EQ2: return of(std::integral_constant<int, FEAT_EQ2>{});
    case FEAT_EQ2 | FEAT_FORCE | FEAT_DRAG:
      return of(std::integral_constant<int, FEAT_EQ2 | FEAT_FORCE | FEAT_DRAG>{});
    case FEAT_MASK | FEAT_SCHEME: return of(std::integral_constant<int, FEAT_MASK | FEAT_SCHEME>{});
    case FEAT_MASK | FEAT_SCHEME | FEAT_FORCE | FEAT_DRAG:
      return of(std::integral_constant<int, FEAT_MASK | FEAT_SCHEME | FEAT_FORCE | FEAT_DRAG>{});
    case FEAT_MASK | FEAT_EQ2: return of(std::integral_constant<int, FEAT_MASK | FEAT_EQ2>{});
    case FEAT_MASK | FEAT_EQ2 | FEAT_FORCE | FEAT_DRAG:
      return of(std::integral_constant<int, FEAT_MASK | FEAT_EQ2 | FEAT_FORCE | FEAT_DRAG>{});
    default: return of(std::integral_constant<int, 0>{});
  }
}

// Two-step workgroups resident per CU: by waves (step2_waves_of per SIMD)
// and by the CU's 160 KB of LDS
int fused_per_cu(const vanse_lattice* h) {
  const int feat = std::max(fused_inst(h), 0);
  unsigned lds = 0;
  switch (h->d.precision) {
    case VANSE_F64: lds = fused_lds_bytes<double, double>(feat); break;
    case VANSE_F16_SHIFTED: lds = fused_lds_bytes<_Float16, float>(feat); break;
    default: lds = fused_lds_bytes<float, float>(feat);
  }
  const int waves = 4 * step2_waves_of(arith_bytes(h), feat) / (2 * fused_nt_of(h) / 64);
  return std::max(1, std::min(waves, int(160u * 1024u / lds)));
}

int fused_rows(const vanse_lattice* h) {
  if (h->rows2 > 0) return h->rows2;
  const int strips = (h->d.nx + fused_out_w(h) - 1) / fused_out_w(h);
  long long nby = (long long)device_cus() * fused_per_cu(h) / strips;
  if (nby < 1) nby = 1;
  long long r = (h->d.ny + nby - 1) / nby;
  if (r < 4) r = 4;
  return (int)r;
}

template <typename S, typename T, bool SHIFT>
int run_fused_pairs(vanse_lattice* h, int64_t pairs, hipStream_t st) {
  const StepPhys<T> ph = make_phys<T>(h);
  const int feat = fused_inst(h);
  StepGeom g{};
  g.phi = h->ws + h->L.phi;
  g.phin = g.phi;
  g.nbr = h->d.has_mask ? h->ws + h->L.nbr : nullptr;
  g.xwalls = 0;
  g.plane = h->L.plane;
  g.nx = h->d.nx;
  g.ny = h->d.ny;
  g.pitch = h->L.pitch;
  g.out_w = fused_out_w(h);
  g.strips = (h->d.nx + g.out_w - 1) / g.out_w;
  g.rows = fused_rows(h);
  const int blocks = g.strips * ((h->d.ny + g.rows - 1) / g.rows);
  const bool walls = h->d.bc_y == VANSE_WALL;
  for (int64_t s = 0; s < pairs; ++s) {
    g.src = h->ws + h->L.pop[h->cur];
    g.dst = h->ws + h->L.pop[h->cur ^ 1];
    g.phi = h->ws + h->L.phi;
    g.beta = h->d.has_drag ? h->ws + h->L.beta : nullptr;
    g.fxf = h->d.has_force_field ? h->ws + h->L.fx : nullptr;
    g.fyf = h->d.has_force_field ? h->ws + h->L.fy : nullptr;
    // a moving phi: the two pending void fractions, or phi held constant;
    // the second step's force field and drag, or the first step's
    g.phin = h->phin2_set ? h->ws + h->L.phin : g.phi;
    g.phin2 = h->phin2_set ? h->ws + h->L.phin2 : g.phi;
    g.beta2 = (h->phin2_set && h->beta2_set) ? h->ws + h->L.beta2 : g.beta;
    g.fxf2 = (h->phin2_set && h->f2_set) ? h->ws + h->L.fx2 : g.fxf;
    g.fyf2 = (h->phin2_set && h->f2_set) ? h->ws + h->L.fy2 : g.fyf;
    auto with_walls = [&](auto feat_c) {
      constexpr int F = decltype(feat_c)::value;
      if (walls) launch_step2<S, T, SHIFT, true, F>(g, ph, blocks, st);
      else launch_step2<S, T, SHIFT, false, F>(g, ph, blocks, st);
    };
    switch (feat) {
      case FEAT_DRAG: with_walls(std::integral_constant<int, FEAT_DRAG>{}); break;
      case FEAT_FORCE: with_walls(std::integral_constant<int, FEAT_FORCE>{}); break;
      case FEAT_FORCE | FEAT_DRAG: with_walls(std::integral_constant<int, FEAT_FORCE | FEAT_DRAG>{}); break;
      case FEAT_MASK: with_walls(std::integral_constant<int, FEAT_MASK>{}); break;
      case FEAT_MASK | FEAT_DRAG: with_walls(std::integral_constant<int, FEAT_MASK | FEAT_DRAG>{}); break;
      case FEAT_MASK | FEAT_FORCE | FEAT_DRAG:
        with_walls(std::integral_constant<int, FEAT_MASK | FEAT_FORCE | FEAT_DRAG>{});
        break;
      case FEAT_DYNPHI: with_walls(std::integral_constant<int, FEAT_DYNPHI>{}); break;
      case FEAT_DYNPHI | FEAT_DRAG: with_walls(std::integral_constant<int, FEAT_DYNPHI | FEAT_DRAG>{}); break;
      case FEAT_DYNPHI | FEAT_FORCE | FEAT_DRAG:
        with_walls(std::integral_constant<int, FEAT_DYNPHI | FEAT_FORCE | FEAT_DRAG>{});
        break;
      case FEAT_SCHEME: with_walls(std::integral_constant<int, FEAT_SCHEME>{}); break;
      case FEAT_SCHEME | FEAT_DRAG: with_walls(std::integral_constant<int, FEAT_SCHEME | FEAT_DRAG>{}); break;
      case FEAT_SCHEME | FEAT_FORCE | FEAT_DRAG:
        with_walls(std::integral_constant<int, FEAT_SCHEME | FEAT_FORCE | FEAT_DRAG>{});
        break;
      case FEAT_EQ2: with_walls(std::integral_constant<int, FEAT_EQ2>{}); break;
      case FEAT_EQ2 | FEAT_FORCE | FEAT_DRAG:
        with_walls(std::integral_constant<int, FEAT_EQ2 | FEAT_FORCE | FEAT_DRAG>{});
        break;
      case FEAT_MASK | FEAT_SCHEME: with_walls(std::integral_constant<int, FEAT_MASK | FEAT_SCHEME>{}); break;
      case FEAT_MASK | FEAT_SCHEME | FEAT_FORCE | FEAT_DRAG:
        with_walls(std::integral_constant<int, FEAT_MASK | FEAT_SCHEME | FEAT_FORCE | FEAT_DRAG>{});
        break;
      case FEAT_MASK | FEAT_EQ2: with_walls(std::integral_constant<int, FEAT_MASK | FEAT_EQ2>{}); break;
      case FEAT_MASK | FEAT_EQ2 | FEAT_FORCE | FEAT_DRAG:
        with_walls(std::integral_constant<int, FEAT_MASK | FEAT_EQ2 | FEAT_FORCE | FEAT_DRAG>{});
        break;
      default: with_walls(std::integral_constant<int, 0>{});
    }
    h->cur ^= 1;
    h->t += 2;
    if (h->phin2_set) {  // the second step's inputs become the current ones
      std::swap(h->L.phi, h->L.phin2);
      if (h->beta2_set) std::swap(h->L.beta, h->L.beta2);
      if (h->f2_set) {
        std::swap(h->L.fx, h->L.fx2);
        std::swap(h->L.fy, h->L.fy2);
      }
      h->phin2_set = h->beta2_set = h->f2_set = false;
      h->version += 1;
    }
    if (s == 0) HIP_TRY(hipGetLastError());
  }
  return VANSE_OK;
}

template <typename S, typename T, bool SHIFT>
int run_steps(vanse_lattice* h, int64_t n, hipStream_t st) {
  if (h->phin_set && n > 1)
    return fail(VANSE_ERR_INVALID_ARG, "with phi(t+1) set, a call advances one step (asked for %lld)", (long long)n);
  if (h->phin2_set && n > 2)
    return fail(VANSE_ERR_INVALID_ARG, "with phi(t+1) and phi(t+2) set, a call advances at most two steps "
                "(asked for %lld)", (long long)n);
  if (fused_ok(h) && n >= 2 && !h->phin_set) {
    if (int rc = run_fused_pairs<S, T, SHIFT>(h, n / 2, st)) return rc;
    n &= 1;
    if (n == 0) return VANSE_OK;
  }
  if (h->phin2_set) {
    // one step at a time: phi(t+1) takes the one-step path of a pending
    // void fraction, and the second step's inputs follow it (below)
    h->phin_set = true;
  }
  const StepPhys<T> ph = make_phys<T>(h);
  StepGeom g{};
  g.nbr = h->d.has_mask ? h->ws + h->L.nbr : nullptr;
  g.xwalls = h->d.bc_x == VANSE_WALL;
  g.plane = h->L.plane;
  g.nx = h->d.nx;
  g.ny = h->d.ny;
  g.pitch = h->L.pitch;
  g.out_w = h->threads - 4;
  g.strips = (h->d.nx + g.out_w - 1) / g.out_w;
  g.rows = h->rows;
  const int nby = (h->d.ny + g.rows - 1) / g.rows;
  const int blocks = g.strips * nby;
  for (int64_t s = 0; s < n; ++s) {
    g.src = h->ws + h->L.pop[h->cur];
    g.dst = h->ws + h->L.pop[h->cur ^ 1];
    g.phi = h->ws + h->L.phi;
    g.phin = h->phin_set ? h->ws + h->L.phin : g.phi;
    g.fxf = h->d.has_force_field ? h->ws + h->L.fx : nullptr;
    g.fyf = h->d.has_force_field ? h->ws + h->L.fy : nullptr;
    g.beta = h->d.has_drag ? h->ws + h->L.beta : nullptr;
    const int rc = by_variant(h, [&](auto walls, auto feat) -> int {
      return launch_step_w<S, T, SHIFT, decltype(walls)::value, decltype(feat)::value>(h, g, ph, blocks, st);
    });
    if (rc != VANSE_OK) return rc;
    h->cur ^= 1;
    h->t += 1;
    if (h->phin_set) {  // phi(t+1) becomes the current void fraction
      std::swap(h->L.phi, h->L.phin);
      h->phin_set = false;
      h->version += 1;
    }
    if (h->phin2_set) {
      // the first of two pending steps is done: phi(t+2) is pending as the
      // next phi(t+1), with the second step's force field and drag
      std::swap(h->L.phin, h->L.phin2);
      if (h->beta2_set) std::swap(h->L.beta, h->L.beta2);
      if (h->f2_set) {
        std::swap(h->L.fx, h->L.fx2);
        std::swap(h->L.fy, h->L.fy2);
      }
      h->phin2_set = h->beta2_set = h->f2_set = false;
      h->phin_set = true;
    }
    if (s == 0) HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipGetLastError());
  return VANSE_OK;
}

// Dispatch on the storage precision: F(S, T, SHIFT) is a generic lambda.
template <typename Fn>
int by_precision(const vanse_lattice* h, Fn&& fn) {
  switch (h->d.precision) {
    case VANSE_F64: return fn((double*)nullptr, (double*)nullptr, std::false_type{});
    case VANSE_F32: return fn((float*)nullptr, (float*)nullptr, std::false_type{});
    case VANSE_F32_SHIFTED: return fn((float*)nullptr, (float*)nullptr, std::true_type{});
    case VANSE_F16_SHIFTED: return fn((_Float16*)nullptr, (float*)nullptr, std::true_type{});
  }
  return fail(VANSE_ERR_INVALID_ARG, "unknown precision");
}

int check_handle(const vanse_lattice* h) {
  if (!h) return fail(VANSE_ERR_INVALID_ARG, "handle is NULL");
  return VANSE_OK;
}

int check_ready(const vanse_lattice* h) {
  if (int rc = check_handle(h)) return rc;
  if (!h->phi_set) return fail(VANSE_ERR_STATE, "void fraction not set");
  if (!h->params_set) return fail(VANSE_ERR_STATE, "kappa and rates not set");
  if (h->d.has_force_field && !h->ff_set) return fail(VANSE_ERR_STATE, "force field not set");
  if (h->d.has_drag && !h->drag_set) return fail(VANSE_ERR_STATE, "drag field not set");
  if (h->d.has_mask && !h->mask_set) return fail(VANSE_ERR_STATE, "mask not set");
  return VANSE_OK;
}

dim3 field_grid(const vanse_lattice* h) { return dim3((h->d.nx + 255) / 256, h->d.ny); }

}  // namespace

// Scratch of vanse_observe_noalloc: the FP64 block partials of one read-out
// (one record per 256-column block of a row, at most kScratchBlocks), the
// chunk records of the first reduction level and the final record.  Each
// device holds its own copy for the life of the process; every call on a
// device overwrites it, so calls that overlap on one device race.
constexpr long long kScratchBlocks = 1LL << 17;
static __device__ __align__(256) double scratch[(kScratchBlocks + 1024 + 1) * NOBS];

namespace {

// Device address of `scratch` on the current device, looked up once per
// device (the array's name in host code is a host-side stand-in, not a
// device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_addr[kMaxDevices] = {};

int scratch_of_device(double** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(VANSE_ERR_HIP, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(VANSE_ERR_HIP, "hipGetSymbolAddress returned no address");
    g_scratch_addr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_addr[dev];
  return VANSE_OK;
}

}  // namespace

extern "C" {

int vanse_workspace_bytes(const vanse_desc* d, size_t* bytes) {
  if (!bytes) return fail(VANSE_ERR_INVALID_ARG, "bytes is NULL");
  Layout L;
  if (int rc = make_layout(d, &L)) return rc;
  *bytes = L.total;
  return VANSE_OK;
}

int vanse_create(const vanse_desc* d, void* workspace, size_t bytes, vanse_lattice** out) {
  if (!out) return fail(VANSE_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  Layout L;
  if (int rc = make_layout(d, &L)) return rc;
  if (!workspace) return fail(VANSE_ERR_WORKSPACE, "workspace is NULL");
  if (((uintptr_t)workspace) & 255) return fail(VANSE_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < L.total) return fail(VANSE_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", bytes, L.total);
  vanse_lattice* h = new (std::nothrow) vanse_lattice();
  if (!h) return fail(VANSE_ERR_INVALID_ARG, "out of host memory");
  h->d = *d;
  h->L = L;
  h->ws = static_cast<char*>(workspace);
  h->cur = 0;
  h->t = 0;
  h->phi_set = h->params_set = h->state_set = h->ff_set = h->drag_set = h->uprev_valid = false;
  h->mask_set = h->phin_set = false;
  h->phin2_set = h->f2_set = h->beta2_set = false;
  h->usx = h->usy = 0.0;
  h->kappa = 0.5;
  h->rho0 = 1.0;
  h->gx = h->gy = 0.0;
  h->scale_by_phi = 1;
  h->model_b = h->eq2 = 0;
  h->uw_lo = h->uw_hi = 0.0;
  h->nee_lo = h->nee_hi = 0;
  h->un_lo = h->un_hi = 0.0;
  h->rates = vanse_rates{1.0, 1.2, 1.2, 1.2, 1.2};
  h->storage_exp = 12;
  h->version = 0;
  h->tiling_default = true;
  default_tiling(h);
  h->fuse = 1;
  h->rows2 = 0;
  h->check_every = 0;
  *out = h;
  return VANSE_OK;
}

int vanse_destroy(vanse_lattice* h) {
  delete h;
  return VANSE_OK;
}

int vanse_set_params(vanse_lattice* h, double kappa, const vanse_rates* r) {
  if (int rc = check_handle(h)) return rc;
  if (!r) return fail(VANSE_ERR_INVALID_ARG, "rates is NULL");
  if (!(kappa >= 0.0 && kappa <= 1.0)) return fail(VANSE_ERR_INVALID_ARG, "kappa must be in [0, 1] (got %g)", kappa);
  const double s[5] = {r->s_c, r->s_e, r->s_eps, r->s_q, r->s_nu};
  for (double v : s)
    if (!(v > 0.0 && v < 2.0)) return fail(VANSE_ERR_INVALID_ARG, "relaxation rates must be in (0, 2) (got %g)", v);
  h->kappa = kappa;
  h->rates = *r;
  h->params_set = true;
  h->version += 1;
  return VANSE_OK;
}

int vanse_set_scheme(vanse_lattice* h, int model, int equilibrium_order) {
  if (int rc = check_handle(h)) return rc;
  if (model != VANSE_MODEL_A && model != VANSE_MODEL_B) return fail(VANSE_ERR_INVALID_ARG, "unknown model %d", model);
  if (equilibrium_order != 2 && equilibrium_order != 3)
    return fail(VANSE_ERR_INVALID_ARG, "equilibrium order must be 2 or 3 (got %d)", equilibrium_order);
  if (h->state_set) return fail(VANSE_ERR_STATE, "the scheme must be chosen before the populations");
  h->model_b = model == VANSE_MODEL_B;
  h->eq2 = equilibrium_order == 2;
  h->version += 1;
  return VANSE_OK;
}

int vanse_set_wall_velocity(vanse_lattice* h, double u_lo, double u_hi) {
  if (int rc = check_handle(h)) return rc;
  if (h->d.bc_y != VANSE_WALL) return fail(VANSE_ERR_STATE, "the lattice has no walls");
  if (!std::isfinite(u_lo) || !std::isfinite(u_hi)) return fail(VANSE_ERR_INVALID_ARG, "wall velocities must be finite");
  if (h->state_set) return fail(VANSE_ERR_STATE, "wall velocities must be set before the populations");
  if ((h->nee_lo && u_lo != 0.0) || (h->nee_hi && u_hi != 0.0))
    return fail(VANSE_ERR_INVALID_ARG, "a face with a velocity row takes no half-way wall velocity");
  h->uw_lo = u_lo;
  h->uw_hi = u_hi;
  h->version += 1;
  return VANSE_OK;
}

int vanse_set_velocity_rows(vanse_lattice* h, int faces, double u_lo, double u_hi) {
  if (int rc = check_handle(h)) return rc;
  if (faces < 0 || faces > (VANSE_FACE_LO | VANSE_FACE_HI))
    return fail(VANSE_ERR_INVALID_ARG, "faces must be a combination of VANSE_FACE_LO and VANSE_FACE_HI");
  if (h->d.bc_y != VANSE_WALL) return fail(VANSE_ERR_STATE, "the lattice has no walls");
  if (h->d.bc_x != VANSE_PERIODIC || h->d.has_mask)
    return fail(VANSE_ERR_UNSUPPORTED, "velocity rows are built for lattices periodic in x without solid nodes");
  if (h->d.ny < 3) return fail(VANSE_ERR_INVALID_ARG, "velocity rows need ny >= 3 (got %d)", h->d.ny);
  if (!std::isfinite(u_lo) || !std::isfinite(u_hi)) return fail(VANSE_ERR_INVALID_ARG, "velocities must be finite");
  if (h->state_set) return fail(VANSE_ERR_STATE, "velocity rows must be set before the populations");
  const int lo = (faces & VANSE_FACE_LO) ? 1 : 0, hi = (faces & VANSE_FACE_HI) ? 1 : 0;
  if ((lo && h->uw_lo != 0.0) || (hi && h->uw_hi != 0.0))
    return fail(VANSE_ERR_INVALID_ARG, "a face with a half-way wall velocity cannot be a velocity row");
  h->nee_lo = lo;
  h->nee_hi = hi;
  h->un_lo = lo ? u_lo : 0.0;
  h->un_hi = hi ? u_hi : 0.0;
  h->version += 1;
  return VANSE_OK;
}

int vanse_set_body_force(vanse_lattice* h, double gx, double gy, int scale_by_phi) {
  if (int rc = check_handle(h)) return rc;
  if (!std::isfinite(gx) || !std::isfinite(gy)) return fail(VANSE_ERR_INVALID_ARG, "G must be finite");
  if (scale_by_phi != 0 && scale_by_phi != 1) return fail(VANSE_ERR_INVALID_ARG, "scale_by_phi must be 0 or 1");
  h->gx = gx;
  h->gy = gy;
  h->scale_by_phi = scale_by_phi;
  h->version += 1;
  return VANSE_OK;
}

// Check a dense phi field (solid nodes excepted) and convert it into the
// plane at workspace offset `off`; solid nodes get the placeholder phi = 1.
static int upload_phi(vanse_lattice* h, const double* phi, size_t off, hipStream_t st) {
  unsigned long long* bad = reinterpret_cast<unsigned long long*>(h->ws + h->L.badcount);
  HIP_TRY(hipMemsetAsync(bad, 0, sizeof(*bad), st));
  const long long n = (long long)h->d.nx * h->d.ny;
  const uint16_t* nbr = h->mask_set ? (const uint16_t*)(h->ws + h->L.nbr) : nullptr;
  hipLaunchKernelGGL(count_bad_phi, dim3(256), dim3(256), 0, st, phi, h->d.nx, n, nbr, h->L.pitch, bad);
  HIP_TRY(hipGetLastError());
  unsigned long long nbad = 0;
  HIP_TRY(hipMemcpyAsync(&nbad, bad, sizeof(nbad), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (nbad) return fail(VANSE_ERR_INVALID_ARG, "%llu void-fraction values outside (0, 1]", nbad);
  void* dst = h->ws + off;
  const Geo G = make_geo(h);
  if (h->d.precision == VANSE_F64) {
    hipLaunchKernelGGL(convert_field<double>, field_grid(h), dim3(256), 0, st, phi, (double*)dst, h->d.nx, h->d.ny, h->L.pitch);
    if (nbr) hipLaunchKernelGGL(phi_on_solids<double>, field_grid(h), dim3(256), 0, st, G, (double*)dst, nbr);
  } else {
    hipLaunchKernelGGL(convert_field<float>, field_grid(h), dim3(256), 0, st, phi, (float*)dst, h->d.nx, h->d.ny, h->L.pitch);
    if (nbr) hipLaunchKernelGGL(phi_on_solids<float>, field_grid(h), dim3(256), 0, st, G, (float*)dst, nbr);
  }
  HIP_TRY(hipGetLastError());
  return VANSE_OK;
}

int vanse_set_void_fraction(vanse_lattice* h, const double* phi, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!phi) return fail(VANSE_ERR_INVALID_ARG, "phi is NULL");
  if (h->phin_set || h->phin2_set) return fail(VANSE_ERR_STATE, "phi(t+1) is pending; step first");
  if (int rc = upload_phi(h, phi, h->L.phi, static_cast<hipStream_t>(stream))) return rc;
  h->phi_set = true;
  h->version += 1;
  return VANSE_OK;
}

int vanse_set_void_fraction_next(vanse_lattice* h, const double* phi_next, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!h->d.dynamic_phi) return fail(VANSE_ERR_STATE, "lattice was created without dynamic_phi");
  if (!phi_next) return fail(VANSE_ERR_INVALID_ARG, "phi_next is NULL");
  if (!h->phi_set) return fail(VANSE_ERR_STATE, "void fraction not set");
  if (h->phin2_set) return fail(VANSE_ERR_STATE, "phi(t+1) and phi(t+2) are pending; step first");
  if (int rc = upload_phi(h, phi_next, h->L.phin, static_cast<hipStream_t>(stream))) return rc;
  h->phin_set = true;
  h->version += 1;
  return VANSE_OK;
}

int vanse_set_void_fraction_next2(vanse_lattice* h, const double* phi_next, const double* phi_next2,
                                  const double* beta_next, const double* fx_next, const double* fy_next,
                                  void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!h->d.dynamic_phi) return fail(VANSE_ERR_STATE, "lattice was created without dynamic_phi");
  if (!phi_next || !phi_next2) return fail(VANSE_ERR_INVALID_ARG, "phi_next or phi_next2 is NULL");
  if (!h->phi_set) return fail(VANSE_ERR_STATE, "void fraction not set");
  if (h->phin_set || h->phin2_set) return fail(VANSE_ERR_STATE, "a void fraction is pending; step first");
  if (beta_next && !h->d.has_drag) return fail(VANSE_ERR_STATE, "lattice was created without drag");
  if ((fx_next != nullptr) != (fy_next != nullptr))
    return fail(VANSE_ERR_INVALID_ARG, "give both force planes of the second step, or neither");
  if (fx_next && !h->d.has_force_field) return fail(VANSE_ERR_STATE, "lattice was created without a force field");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int rc = upload_phi(h, phi_next, h->L.phin, st)) return rc;
  if (int rc = upload_phi(h, phi_next2, h->L.phin2, st)) return rc;
  const double* in[3] = {beta_next, fx_next, fy_next};
  const size_t off[3] = {h->L.beta2, h->L.fx2, h->L.fy2};
  for (int k = 0; k < 3; ++k) {
    if (!in[k]) continue;
    void* dst = h->ws + off[k];
    if (h->d.precision == VANSE_F64)
      hipLaunchKernelGGL(convert_field<double>, field_grid(h), dim3(256), 0, st, in[k], (double*)dst, h->d.nx, h->d.ny, h->L.pitch);
    else
      hipLaunchKernelGGL(convert_field<float>, field_grid(h), dim3(256), 0, st, in[k], (float*)dst, h->d.nx, h->d.ny, h->L.pitch);
  }
  HIP_TRY(hipGetLastError());
  h->phin2_set = true;
  h->beta2_set = beta_next != nullptr;
  h->f2_set = fx_next != nullptr;
  h->version += 1;
  return VANSE_OK;
}

int vanse_set_mask(vanse_lattice* h, const uint8_t* mask, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!h->d.has_mask) return fail(VANSE_ERR_STATE, "lattice was created without a mask");
  if (!mask) return fail(VANSE_ERR_INVALID_ARG, "mask is NULL");
  if (h->state_set) return fail(VANSE_ERR_STATE, "the mask must be set before the populations");
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(h->ws + h->L.badcount);
  HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(*cnt), st));
  const Geo G = make_geo(h);
  uint16_t* nbr = (uint16_t*)(h->ws + h->L.nbr);
  hipLaunchKernelGGL(build_nbr, field_grid(h), dim3(256), 0, st, G, mask, nbr, cnt);
  HIP_TRY(hipGetLastError());
  unsigned long long nsolid = 0;
  HIP_TRY(hipMemcpyAsync(&nsolid, cnt, sizeof(nsolid), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (nsolid == (unsigned long long)h->d.nx * h->d.ny) return fail(VANSE_ERR_INVALID_ARG, "every node is solid");
  if (h->phi_set) {  // placeholder phi on the solid nodes
    if (h->d.precision == VANSE_F64)
      hipLaunchKernelGGL(phi_on_solids<double>, field_grid(h), dim3(256), 0, st, G, (double*)(h->ws + h->L.phi), (const uint16_t*)nbr);
    else
      hipLaunchKernelGGL(phi_on_solids<float>, field_grid(h), dim3(256), 0, st, G, (float*)(h->ws + h->L.phi), (const uint16_t*)nbr);
    HIP_TRY(hipGetLastError());
  }
  h->mask_set = true;
  h->version += 1;
  return VANSE_OK;
}

int vanse_set_force_field(vanse_lattice* h, const double* fx, const double* fy, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!h->d.has_force_field) return fail(VANSE_ERR_STATE, "lattice was created without a force field");
  if (!fx || !fy) return fail(VANSE_ERR_INVALID_ARG, "force planes are NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double* in[2] = {fx, fy};
  const size_t off[2] = {h->L.fx, h->L.fy};
  for (int k = 0; k < 2; ++k) {
    void* dst = h->ws + off[k];
    if (h->d.precision == VANSE_F64)
      hipLaunchKernelGGL(convert_field<double>, field_grid(h), dim3(256), 0, st, in[k], (double*)dst, h->d.nx, h->d.ny, h->L.pitch);
    else
      hipLaunchKernelGGL(convert_field<float>, field_grid(h), dim3(256), 0, st, in[k], (float*)dst, h->d.nx, h->d.ny, h->L.pitch);
  }
  HIP_TRY(hipGetLastError());
  h->ff_set = true;
  return VANSE_OK;
}

int vanse_set_drag(vanse_lattice* h, const double* beta, double usx, double usy, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!h->d.has_drag) return fail(VANSE_ERR_STATE, "lattice was created without drag");
  if (!beta) return fail(VANSE_ERR_INVALID_ARG, "beta is NULL");
  if (!std::isfinite(usx) || !std::isfinite(usy)) return fail(VANSE_ERR_INVALID_ARG, "u_s must be finite");
  hipStream_t st = static_cast<hipStream_t>(stream);
  void* dst = h->ws + h->L.beta;
  if (h->d.precision == VANSE_F64)
    hipLaunchKernelGGL(convert_field<double>, field_grid(h), dim3(256), 0, st, beta, (double*)dst, h->d.nx, h->d.ny, h->L.pitch);
  else
    hipLaunchKernelGGL(convert_field<float>, field_grid(h), dim3(256), 0, st, beta, (float*)dst, h->d.nx, h->d.ny, h->L.pitch);
  HIP_TRY(hipGetLastError());
  h->usx = usx;
  h->usy = usy;
  h->drag_set = true;
  h->version += 1;
  return VANSE_OK;
}

static int fill(vanse_lattice* h, const double* fin, double rho0, double ux0, double uy0, void* stream) {
  if (int rc = check_ready(h)) return rc;
  if (!(rho0 > 0.0) || !std::isfinite(rho0)) return fail(VANSE_ERR_INVALID_ARG, "rho0 must be positive");
  hipStream_t st = static_cast<hipStream_t>(stream);
  h->rho0 = rho0;
  const Geo G = make_geo(h);
  const int rc = by_precision(h, [&](auto* s_tag, auto* t_tag, auto shift) -> int {
    using S = std::remove_pointer_t<decltype(s_tag)>;
    using T = std::remove_pointer_t<decltype(t_tag)>;
    constexpr bool SH = decltype(shift)::value;
    const StepPhys<T> ph = make_phys<T>(h);
    const uint16_t* nbr = h->d.has_mask ? (const uint16_t*)(h->ws + h->L.nbr) : nullptr;
    hipLaunchKernelGGL((fill_state<S, T, SH>), field_grid(h), dim3(256), 0, st, G,
                       (S*)(h->ws + h->L.pop[0]), (const T*)(h->ws + h->L.phi), ph, fin, rho0, ux0,
                       uy0, h->kappa, nbr);
    return VANSE_OK;
  });
  if (rc) return rc;
  HIP_TRY(hipGetLastError());
  h->cur = 0;
  h->t = 0;
  h->state_set = true;
  h->uprev_valid = false;
  h->version += 1;
  return VANSE_OK;
}

int vanse_init_equilibrium(vanse_lattice* h, double rho0, double ux0, double uy0, void* stream) {
  if (!std::isfinite(ux0) || !std::isfinite(uy0)) return fail(VANSE_ERR_INVALID_ARG, "u0 must be finite");
  return fill(h, nullptr, rho0, ux0, uy0, stream);
}

int vanse_set_populations(vanse_lattice* h, const double* f, double rho0, void* stream) {
  if (!f) return fail(VANSE_ERR_INVALID_ARG, "populations are NULL");
  return fill(h, f, rho0, 0.0, 0.0, stream);
}

static int moments(vanse_lattice* h, double* rho, double* ux, double* uy, double* p, bool partials,
                   void* stream, bool keep_u = false);
static int reduce_on_device(vanse_lattice* h, hipStream_t st);

static int advance(vanse_lattice* h, int64_t n, hipStream_t st) {
  return by_precision(h, [&](auto* s_tag, auto* t_tag, auto shift) -> int {
    using S = std::remove_pointer_t<decltype(s_tag)>;
    using T = std::remove_pointer_t<decltype(t_tag)>;
    return run_steps<S, T, decltype(shift)::value>(h, n, st);
  });
}

int vanse_step(vanse_lattice* h, int64_t nsteps, void* stream) {
  if (int rc = check_ready(h)) return rc;
  if (!h->state_set) return fail(VANSE_ERR_STATE, "populations not initialised");
  if (nsteps < 0) return fail(VANSE_ERR_INVALID_ARG, "nsteps must be >= 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (h->check_every <= 0) return advance(h, nsteps, st);
  // Observables at every multiple of check_every: enqueued between the
  // launches, each one's non-finite count folded into a device flag that
  // holds the first time it was seen; one synchronizing read at the end.
  long long* flag = reinterpret_cast<long long*>(h->ws + h->L.check);
  bool checked = false;
  // With two steps per launch a check waits for the end of the launch that
  // reaches the multiple of k (t or t + 1), so that the launches of the call
  // are those of an unchecked call: pairs, and one single step at the end
  // when nsteps is odd.
  const bool pairs = fused_ok(h);
  while (nsteps > 0) {
    const int64_t k = h->check_every;
    int64_t m = std::min<int64_t>(nsteps, k - h->t % k);
    if (pairs && (m & 1) && m < nsteps) m += 1;
    if (int rc = advance(h, m, st)) return rc;
    nsteps -= m;
    if (h->t % k == 0 || (pairs && (h->t - 1) % k == 0 && m > 1)) {
      if (!checked) {
        hipLaunchKernelGGL(set_flag, dim3(1), dim3(64), 0, st, flag, -1LL);
        checked = true;
      }
      if (int rc = moments(h, nullptr, nullptr, nullptr, nullptr, true, stream)) return rc;
      if (int rc = reduce_on_device(h, st)) return rc;
      hipLaunchKernelGGL(note_nonfinite, dim3(1), dim3(64), 0, st,
                         (const double*)(h->ws + h->L.result), (long long)h->t, flag);
      HIP_TRY(hipGetLastError());
    }
  }
  if (!checked) return VANSE_OK;
  long long tbad = -1;
  HIP_TRY(hipMemcpyAsync(&tbad, flag, sizeof(tbad), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (tbad >= 0)
    return fail(VANSE_ERR_DIVERGED, "non-finite values observed at t = %lld (checked every %lld steps)",
                tbad, (long long)h->check_every);
  return VANSE_OK;
}

int vanse_set_check_interval(vanse_lattice* h, int64_t k) {
  if (int rc = check_handle(h)) return rc;
  if (k < 0) return fail(VANSE_ERR_INVALID_ARG, "check interval must be >= 0 (got %lld)", (long long)k);
  h->check_every = k;
  return VANSE_OK;
}

// Macroscopic read-out (rho, u, p; any may be null) and, with `part`, the
// FP64 block partials of the observables into part.  plane: delta rho goes
// through the workspace's scratch plane (two passes), else the second pass
// forms every node's delta rho from its populations (no scratch plane).
static int moments_into(vanse_lattice* h, double* rho, double* ux, double* uy, double* p,
                        double* part, bool plane, hipStream_t st, bool keep_u) {
  if (int rc = check_ready(h)) return rc;
  if (!h->state_set) return fail(VANSE_ERR_STATE, "populations not initialised");
  const Geo G = make_geo(h);
  const int rc = by_precision(h, [&](auto* s_tag, auto* t_tag, auto shift) -> int {
    using S = std::remove_pointer_t<decltype(s_tag)>;
    using T = std::remove_pointer_t<decltype(t_tag)>;
    constexpr bool SH = decltype(shift)::value;
    const StepPhys<T> ph = make_phys<T>(h);
    const S* buf = (const S*)(h->ws + h->L.pop[h->cur]);
    const T* phi = (const T*)(h->ws + h->L.phi);
    T* drho = plane ? (T*)(h->ws + h->L.drho) : nullptr;
    const uint16_t* nbr = h->d.has_mask ? (const uint16_t*)(h->ws + h->L.nbr) : nullptr;
    if (plane)
      hipLaunchKernelGGL((moments_rho<S, T, SH>), field_grid(h), dim3(256), 0, st, G, buf, phi, ph, drho, nbr);
    const T* fx = h->d.has_force_field ? (const T*)(h->ws + h->L.fx) : nullptr;
    const T* fy = h->d.has_force_field ? (const T*)(h->ws + h->L.fy) : nullptr;
    const T* beta = h->d.has_drag ? (const T*)(h->ws + h->L.beta) : nullptr;
    return by_variant(h, [&](auto walls, auto feat) -> int {
      (void)walls;
      T* up = keep_u ? (T*)(h->ws + h->L.uprev) : nullptr;
      hipLaunchKernelGGL((moments_out<S, T, SH, decltype(feat)::value>), field_grid(h), dim3(256), 0, st, G,
                         buf, phi, ph, drho, fx, fy, beta, rho, ux, uy, p, part, up,
                         (int)(keep_u && h->uprev_valid), nbr);
      return VANSE_OK;
    });
  });
  if (rc) return rc;
  HIP_TRY(hipGetLastError());
  return VANSE_OK;
}

static int moments(vanse_lattice* h, double* rho, double* ux, double* uy, double* p, bool partials,
                   void* stream, bool keep_u) {
  double* part = partials ? (double*)(h ? h->ws + h->L.partials : nullptr) : nullptr;
  return moments_into(h, rho, ux, uy, p, part, true, static_cast<hipStream_t>(stream), keep_u);
}

int vanse_read_moments(vanse_lattice* h, double* rho, double* ux, double* uy, double* p, void* stream) {
  if (!rho) return fail(VANSE_ERR_INVALID_ARG, "rho output is NULL");
  return moments(h, rho, ux, uy, p, false, stream, false);
}

int vanse_read_populations(vanse_lattice* h, double* f, void* stream) {
  if (int rc = check_ready(h)) return rc;
  if (!h->state_set) return fail(VANSE_ERR_STATE, "populations not initialised");
  if (!f) return fail(VANSE_ERR_INVALID_ARG, "output is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Geo G = make_geo(h);
  const int rc = by_precision(h, [&](auto* s_tag, auto* t_tag, auto shift) -> int {
    using S = std::remove_pointer_t<decltype(s_tag)>;
    using T = std::remove_pointer_t<decltype(t_tag)>;
    constexpr bool SH = decltype(shift)::value;
    const StepPhys<T> ph = make_phys<T>(h);
    const uint16_t* nbr = h->d.has_mask ? (const uint16_t*)(h->ws + h->L.nbr) : nullptr;
    hipLaunchKernelGGL((read_pops<S, T, SH>), field_grid(h), dim3(256), 0, st, G,
                       (const S*)(h->ws + h->L.pop[h->cur]), (const T*)(h->ws + h->L.phi), ph, f, nbr);
    return VANSE_OK;
  });
  if (rc) return rc;
  HIP_TRY(hipGetLastError());
  return VANSE_OK;
}

// Fixed-order reduction of n block partials (in) to one record (res), through
// at most 1024 chunk records (mid); enqueued only.
static int reduce_blocks(const double* in, long long n, double* mid, double* res, hipStream_t st) {
  // level 1: at most 1024 chunks; level 2: one workgroup
  const long long chunk = (n + 1023) / 1024;
  const long long nchunks = (n + chunk - 1) / chunk;
  hipLaunchKernelGGL(reduce_partials, dim3((unsigned)nchunks), dim3(256), 0, st, in, n, chunk, mid);
  hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(256), 0, st, (const double*)mid, nchunks, nchunks, res);
  HIP_TRY(hipGetLastError());
  return VANSE_OK;
}

// Reduce the block partials of the last moments pass to one record in the
// workspace (enqueued only).
static int reduce_on_device(vanse_lattice* h, hipStream_t st) {
  const long long n = (long long)((h->d.nx + 255) / 256) * h->d.ny;
  return reduce_blocks((const double*)(h->ws + h->L.partials), n, (double*)(h->ws + h->L.partials2),
                       (double*)(h->ws + h->L.result), st);
}

// The same, copied to the host (synchronizes the stream).
static int reduce_to_host(vanse_lattice* h, double* rec, hipStream_t st) {
  if (int rc = reduce_on_device(h, st)) return rc;
  const double* res = (const double*)(h->ws + h->L.result);
  HIP_TRY(hipMemcpyAsync(rec, res, NOBS * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return VANSE_OK;
}

int vanse_observe(vanse_lattice* h, double* out, void* stream) {
  if (!out) return fail(VANSE_ERR_INVALID_ARG, "out is NULL");
  if (int rc = moments(h, nullptr, nullptr, nullptr, nullptr, true, stream, false)) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  double rec[NOBS];
  if (int rc = reduce_to_host(h, rec, st)) return rc;
  for (int q = 0; q < 4; ++q) out[q] = rec[q];
  if (out[3] > 0) return fail(VANSE_ERR_DIVERGED, "%.0f nodes hold non-finite values at t = %lld", out[3], (long long)h->t);
  return VANSE_OK;
}

int vanse_observe_noalloc(vanse_lattice* h, double* out, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!out) return fail(VANSE_ERR_INVALID_ARG, "out is NULL");
  const long long nblk = (long long)((h->d.nx + 255) / 256) * h->d.ny;
  if (nblk > kScratchBlocks)
    return fail(VANSE_ERR_INVALID_ARG,
                "lattice too large for the static scratch: %lld read-out blocks of 256 columns > %lld",
                nblk, kScratchBlocks);
  if (int rc = check_ready(h)) return rc;
  if (!h->state_set) return fail(VANSE_ERR_STATE, "populations not initialised");
  double* sp = nullptr;
  if (int rc = scratch_of_device(&sp)) return rc;
  double* part = sp;
  double* mid = sp + kScratchBlocks * NOBS;
  double* res = mid + 1024 * NOBS;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int rc = moments_into(h, nullptr, nullptr, nullptr, nullptr, part, false, st, false)) return rc;
  if (int rc = reduce_blocks(part, nblk, mid, res, st)) return rc;
  double rec[NOBS];
  HIP_TRY(hipMemcpyAsync(rec, res, NOBS * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int q = 0; q < 4; ++q) out[q] = rec[q];
  if (out[3] > 0) return fail(VANSE_ERR_DIVERGED, "%.0f nodes hold non-finite values at t = %lld", out[3], (long long)h->t);
  return VANSE_OK;
}

int vanse_residual(vanse_lattice* h, double* out, void* stream) {
  if (!out) return fail(VANSE_ERR_INVALID_ARG, "out is NULL");
  const bool had_prev = h && h->uprev_valid;
  if (int rc = moments(h, nullptr, nullptr, nullptr, nullptr, true, stream, true)) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  double rec[NOBS];
  if (int rc = reduce_to_host(h, rec, st)) return rc;
  h->uprev_valid = true;
  out[0] = had_prev ? rec[4] : -1.0;
  out[1] = rec[1];
  out[2] = rec[3];
  if (rec[3] > 0) return fail(VANSE_ERR_DIVERGED, "%.0f nodes hold non-finite values at t = %lld", rec[3], (long long)h->t);
  return VANSE_OK;
}

int vanse_set_tiling(vanse_lattice* h, int threads, int rows) {
  if (int rc = check_handle(h)) return rc;
  if (threads == 0 || rows == 0) {
    h->tiling_default = true;
    default_tiling(h);
    return VANSE_OK;
  }
  if (threads != 64 && threads != 128 && threads != 256 && threads != 512)
    return fail(VANSE_ERR_INVALID_ARG, "threads must be 64, 128, 256 or 512 (got %d)", threads);
  if (rows < 1) return fail(VANSE_ERR_INVALID_ARG, "rows must be >= 1 (got %d)", rows);
  h->threads = threads;
  h->rows = rows;
  h->tiling_default = false;
  return VANSE_OK;
}

int vanse_set_steps_per_pass(vanse_lattice* h, int steps, int rows) {
  if (int rc = check_handle(h)) return rc;
  if (steps != 1 && steps != 2) return fail(VANSE_ERR_INVALID_ARG, "steps per pass must be 1 or 2 (got %d)", steps);
  if (rows < 0) return fail(VANSE_ERR_INVALID_ARG, "rows must be >= 0 (got %d)", rows);
  h->fuse = steps;
  h->rows2 = rows;
  return VANSE_OK;
}

int vanse_get_fused_tiling(const vanse_lattice* h, int* active, int* rows, int* workgroups) {
  if (int rc = check_handle(h)) return rc;
  const int r = fused_rows(h);
  const int strips = (h->d.nx + fused_out_w(h) - 1) / fused_out_w(h);
  if (active) *active = fused_ok(h) ? 1 : 0;
  if (rows) *rows = r;
  if (workgroups) *workgroups = strips * ((h->d.ny + r - 1) / r);
  return VANSE_OK;
}

int vanse_get_tiling(const vanse_lattice* h, int* threads, int* rows, int* workgroups) {
  if (int rc = check_handle(h)) return rc;
  const int out_w = h->threads - 4;
  const int strips = (h->d.nx + out_w - 1) / out_w;
  const int nby = (h->d.ny + h->rows - 1) / h->rows;
  if (threads) *threads = h->threads;
  if (rows) *rows = h->rows;
  if (workgroups) *workgroups = strips * nby;
  return VANSE_OK;
}

int vanse_set_storage_exponent(vanse_lattice* h, int e) {
  if (int rc = check_handle(h)) return rc;
  if (e < -24 || e > 24) return fail(VANSE_ERR_INVALID_ARG, "storage exponent out of range (got %d)", e);
  if (h->state_set) return fail(VANSE_ERR_STATE, "storage exponent must be set before the populations");
  h->storage_exp = e;
  h->version += 1;
  return VANSE_OK;
}

int vanse_stream_copy(vanse_lattice* h, int64_t n, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (n < 0) return fail(VANSE_ERR_INVALID_ARG, "n must be >= 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Geo G = make_geo(h);
  const int sb = storage_bytes(h->d.precision);
  for (int64_t s = 0; s < n; ++s) {
    const void* src = h->ws + h->L.pop[h->cur];
    void* dst = h->ws + h->L.pop[h->cur ^ 1];
    if (sb == 8)
      hipLaunchKernelGGL(stream_copy<double>, field_grid(h), dim3(256), 0, st, G, (const double*)src, (double*)dst);
    else if (sb == 4)
      hipLaunchKernelGGL(stream_copy<float>, field_grid(h), dim3(256), 0, st, G, (const float*)src, (float*)dst);
    else
      hipLaunchKernelGGL(stream_copy<_Float16>, field_grid(h), dim3(256), 0, st, G, (const _Float16*)src, (_Float16*)dst);
    h->cur ^= 1;
  }
  HIP_TRY(hipGetLastError());
  return VANSE_OK;
}

int64_t vanse_time(const vanse_lattice* h) { return h ? h->t : -1; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: many independent lattices advanced by one launch per time step.
// ---------------------------------------------------------------------------
struct vanse_batch {
  std::vector<vanse_lattice*> lats;
  std::vector<int> rows;     // rows per workgroup, per lattice
  std::vector<int> first;    // first tile of each lattice
  int threads = 256;
  int fuse = 1;              // time steps per launch (2: the two-step kernel)
  int total_tiles = 0;
  char* ws = nullptr;
  size_t entries_off = 0, tiles_off = 0;
  bool table_ready = false;
  long long launched = 0;    // launches since the table was written
  std::vector<long long> versions;  // member versions at the last upload
  std::vector<int> cur0;            // member buffer parity at the last upload
  int graph_steps = 0;
  hipGraphExec_t graph = nullptr;
  hipStream_t own = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
};

namespace {

// Resident workgroups per CU: 16 waves per CU in FP32 arithmetic (four per
// SIMD), 8 in FP64; a one-step workgroup has `threads` lanes, a two-step
// one 2 x threads.
int batch_per_cu(int precision, int threads, int fuse) {
  const int waves_per_cu = precision == VANSE_F64 ? 8 : 16;
  return waves_per_cu * 64 / (fuse * threads);
}

// Columns a tile outputs: threads - 4 for one step, threads - 10 for two
int batch_out_w(int threads, int fuse) { return threads - (fuse == 2 ? 10 : 4); }

int batch_layout(vanse_lattice* const* lats, int n, int threads, int rows, int fuse,
                 std::vector<int>* rows_out, std::vector<int>* first_out, int* total_tiles,
                 size_t* entries_off, size_t* tiles_off, size_t* bytes) {
  if (!lats || n < 1) return fail(VANSE_ERR_INVALID_ARG, "a batch needs at least one lattice");
  if (threads != 64 && threads != 128 && threads != 256)
    return fail(VANSE_ERR_INVALID_ARG, "batch threads must be 64, 128 or 256 (got %d)", threads);
  if (rows < 0) return fail(VANSE_ERR_INVALID_ARG, "rows must be >= 0");
  if (fuse != 1 && fuse != 2) return fail(VANSE_ERR_INVALID_ARG, "steps per pass must be 1 or 2 (got %d)", fuse);
  const vanse_desc& d0 = lats[0] ? lats[0]->d : vanse_desc{};
  // two-step halves of at most step2_nt_of lanes (FP64 rings take twice the
  // LDS per lane; solid nodes with the drag two more planes)
  if (fuse == 2 && lats[0] && threads > fused_nt_of(lats[0]))
    return fail(VANSE_ERR_UNSUPPORTED, "%s batches with two steps per launch take at most %d threads",
                d0.precision == VANSE_F64 ? "FP64" : "these", fused_nt_of(lats[0]));
  const int out_w = batch_out_w(threads, fuse);
  long long strip_rows = 0;
  for (int k = 0; k < n; ++k) {
    if (!lats[k]) return fail(VANSE_ERR_INVALID_ARG, "lattice %d is NULL", k);
    const vanse_desc& d = lats[k]->d;
    if (!batch_ok(lats[k]))
      return fail(VANSE_ERR_UNSUPPORTED,
                  "lattice %d: batches take no time-varying phi, velocity rows, nor a scheme variant "
                  "with solid nodes", k);
    if (d.precision != d0.precision || d.bc_x != d0.bc_x || d.bc_y != d0.bc_y ||
        d.has_force_field != d0.has_force_field ||
        d.has_drag != d0.has_drag || feat_of(lats[k]) != feat_of(lats[0]))
      return fail(VANSE_ERR_INVALID_ARG,
                  "lattice %d differs in precision, boundary, force field, drag, mask or scheme variant", k);
    if (fuse == 2 && !fused_feat(lats[k]))
      return fail(VANSE_ERR_UNSUPPORTED,
                  "lattice %d: two steps per launch take the force field, the drag, solid nodes and "
                  "the scheme variants only (no walls in x or wall velocities)", k);
    // (the one-step instance of the scheme variants serves model B and the
    // Appendix B equilibrium alike through run-time flags; the two-step
    // instances do not)
    if (fuse == 2 && fused_inst(lats[k]) != fused_inst(lats[0]))
      return fail(VANSE_ERR_INVALID_ARG, "lattice %d differs in its two-step instance (scheme variant)", k);
    strip_rows += (long long)((d.nx + out_w - 1) / out_w) * d.ny;
  }
  int r = rows;
  if (r == 0) {
    // about two rounds of resident workgroups over the whole batch for one
    // step per launch, four for two (measured on 256 lattices of side 32 to
    // 512: shorter tiles balance the uneven lattices better), but at least
    // 32 rows for two (each two-step tile sweeps 11 rows beyond its own)
    const int rounds = fuse == 2 ? 4 : 2;
    const long long slots = (long long)device_cus() * batch_per_cu(d0.precision, threads, fuse);
    r = (int)((strip_rows + rounds * slots - 1) / (rounds * slots));
    const int rmin = fuse == 2 ? 32 : 8;
    if (r < rmin) r = rmin;
  }
  rows_out->assign(n, r);
  first_out->assign(n, 0);
  long long tiles = 0;
  for (int k = 0; k < n; ++k) {
    const vanse_desc& d = lats[k]->d;
    (*first_out)[k] = (int)tiles;
    tiles += (long long)((d.nx + out_w - 1) / out_w) * ((d.ny + r - 1) / r);
  }
  if (tiles > (1LL << 30)) return fail(VANSE_ERR_INVALID_ARG, "too many tiles");
  *total_tiles = (int)tiles;
  const size_t esz = sizeof(BatchEntry<double>) > sizeof(BatchEntry<float>) ? sizeof(BatchEntry<double>)
                                                                            : sizeof(BatchEntry<float>);
  *entries_off = 0;
  *tiles_off = align256((size_t)n * esz);
  // then one FP64 observables record per member (vanse_batch_residual)
  *bytes = align256(align256(*tiles_off + (size_t)tiles * sizeof(int2)) + (size_t)n * NOBS * sizeof(double));
  return VANSE_OK;
}

template <typename T>
void fill_entries(vanse_batch* b, std::vector<char>* blob) {
  const int n = (int)b->lats.size();
  blob->assign((size_t)n * sizeof(BatchEntry<T>), 0);
  BatchEntry<T>* E = reinterpret_cast<BatchEntry<T>*>(blob->data());
  for (int k = 0; k < n; ++k) {
    vanse_lattice* h = b->lats[k];
    StepGeom g;
    g.src = h->ws + h->L.pop[0];
    g.dst = h->ws + h->L.pop[1];
    g.phi = h->ws + h->L.phi;
    g.phin = g.phi;
    g.nbr = h->d.has_mask ? h->ws + h->L.nbr : nullptr;
    g.xwalls = h->d.bc_x == VANSE_WALL;
    g.fxf = h->d.has_force_field ? h->ws + h->L.fx : nullptr;
    g.fyf = h->d.has_force_field ? h->ws + h->L.fy : nullptr;
    g.beta = h->d.has_drag ? h->ws + h->L.beta : nullptr;
    g.plane = h->L.plane;
    g.nx = h->d.nx;
    g.ny = h->d.ny;
    g.pitch = h->L.pitch;
    g.out_w = batch_out_w(b->threads, b->fuse);
    g.strips = (h->d.nx + g.out_w - 1) / g.out_w;
    g.rows = b->rows[k];
    E[k].g = g;
    E[k].ph = make_phys<T>(h);
    E[k].first_tile = b->first[k];
    E[k].cur0 = h->cur;
  }
}

// Tile map of a batch: for every tile position, the lattice and the tile's
// index within it.  Workgroup b reads position xcd_tile(b): the workgroups
// dealt to XCD x read the x-th contiguous run of positions, in order.  The
// tiles are laid out lattice by lattice (strips side by side, so that
// neighbouring strips, which read each other's halo columns, share the
// XCD's L2), and each XCD's run is then ordered by decreasing sweep length
// (rows of the tile: a lattice's last row block may be short), ties in
// lattice order: the short tiles fill the tail of the launch
// (longest-processing-time-first list scheduling on every XCD).
std::vector<int2> batch_tile_map(const vanse_batch* b) {
  struct Item { int rows, k, local; };
  std::vector<Item> items;
  items.reserve((size_t)b->total_tiles);
  const int out_w = batch_out_w(b->threads, b->fuse);
  for (size_t k = 0; k < b->lats.size(); ++k) {
    const vanse_desc& d = b->lats[k]->d;
    const int r = b->rows[k];
    const int strips = (d.nx + out_w - 1) / out_w;
    const int nby = (d.ny + r - 1) / r;
    for (int local = 0; local < strips * nby; ++local) {
      const int by = local / strips;
      items.push_back({std::min(r, d.ny - by * r), (int)k, local});
    }
  }
  const int nb = b->total_tiles, q = nb >> 3, rem = nb & 7;
  for (int x = 0; x < 8; ++x) {  // the run of XCD x, as in xcd_tile
    const int s0 = x * q + std::min(x, rem), s1 = s0 + q + (x < rem ? 1 : 0);
    std::stable_sort(items.begin() + s0, items.begin() + s1,
                     [](const Item& a, const Item& c) { return a.rows > c.rows; });
  }
  std::vector<int2> map((size_t)nb);
  for (int i = 0; i < nb; ++i) map[(size_t)i] = make_int2(items[(size_t)i].k, items[(size_t)i].local);
  return map;
}

// Upload the lattice table and the tile map (host pageable copies,
// synchronized: only when parameters or buffer parity change).
int batch_upload(vanse_batch* b, hipStream_t st) {
  std::vector<char> blob;
  if (b->lats[0]->d.precision == VANSE_F64) fill_entries<double>(b, &blob);
  else fill_entries<float>(b, &blob);
  const std::vector<int2> tl = batch_tile_map(b);
  HIP_TRY(hipMemcpyAsync(b->ws + b->entries_off, blob.data(), blob.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(b->ws + b->tiles_off, tl.data(), tl.size() * sizeof(int2), hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  b->versions.resize(b->lats.size());
  b->cur0.resize(b->lats.size());
  for (size_t k = 0; k < b->lats.size(); ++k) {
    b->versions[k] = b->lats[k]->version;
    b->cur0[k] = b->lats[k]->cur;
  }
  b->table_ready = true;
  b->launched = 0;
  return VANSE_OK;
}

template <typename S, typename T, bool SHIFT, bool WALLS, int FEAT>
int batch_launch_t(vanse_batch* b, int launch, hipStream_t st) {
  const BatchEntry<T>* E = reinterpret_cast<const BatchEntry<T>*>(b->ws + b->entries_off);
  const int2* TL = reinterpret_cast<const int2*>(b->ws + b->tiles_off);
  if constexpr ((FEAT & ~(FEAT_FORCE | FEAT_DRAG | FEAT_MASK | FEAT_SCHEME | FEAT_EQ2)) == 0) {
    if (b->fuse == 2) {
      // halves of 64 up to step2_nt_of lanes (batch_layout)
      if (!launch_batch2<S, T, SHIFT, WALLS, FEAT>(b->threads, E, TL, launch, b->total_tiles, st))
        return fail(VANSE_ERR_UNSUPPORTED, "no two-step batch kernel with halves of %d lanes", b->threads);
      return VANSE_OK;
    }
  }
  if constexpr (FEAT == (FEAT_MASK | FEAT_DRAG) || FEAT == FEAT_SCHEME || FEAT == (FEAT_SCHEME | FEAT_DRAG) ||
                FEAT == (FEAT_SCHEME | FEAT_FORCE | FEAT_DRAG) || (FEAT & FEAT_EQ2) != 0) {
    // a two-step instance only (one step per launch takes FEAT_MASK |
    // FEAT_FORCE | FEAT_DRAG, or FEAT_SCHEME | FEAT_MOVING): no one-step
    // batch kernel is built for it
    return fail(VANSE_ERR_UNSUPPORTED, "no one-step batch kernel of this variant");
  } else {
    switch (b->threads) {
      case 64: launch_batch_nt<S, T, SHIFT, WALLS, FEAT, 64>(E, TL, launch, b->total_tiles, st); break;
      case 128: launch_batch_nt<S, T, SHIFT, WALLS, FEAT, 128>(E, TL, launch, b->total_tiles, st); break;
      default: launch_batch_nt<S, T, SHIFT, WALLS, FEAT, 256>(E, TL, launch, b->total_tiles, st);
    }
    return VANSE_OK;
  }
}

int batch_launch(vanse_batch* b, int launch, hipStream_t st) {
  return by_precision(b->lats[0], [&](auto* s_tag, auto* t_tag, auto shift) -> int {
    using S = std::remove_pointer_t<decltype(s_tag)>;
    using T = std::remove_pointer_t<decltype(t_tag)>;
    constexpr bool SH = decltype(shift)::value;
    if (b->fuse == 2) {  // the two-step instances that are no one-step variant (see fused_inst)
      const bool walls = b->lats[0]->d.bc_y == VANSE_WALL;
      auto go = [&](auto feat) -> int {
        constexpr int F = decltype(feat)::value;
        return walls ? batch_launch_t<S, T, SH, true, F>(b, launch, st)
                     : batch_launch_t<S, T, SH, false, F>(b, launch, st);
      };
      switch (fused_inst(b->lats[0])) {
        case FEAT_MASK | FEAT_DRAG: return go(std::integral_constant<int, FEAT_MASK | FEAT_DRAG>{});
        case FEAT_SCHEME: return go(std::integral_constant<int, FEAT_SCHEME>{});
        case FEAT_SCHEME | FEAT_DRAG: return go(std::integral_constant<int, FEAT_SCHEME | FEAT_DRAG>{});
        case FEAT_SCHEME | FEAT_FORCE | FEAT_DRAG:
          return go(std::integral_constant<int, FEAT_SCHEME | FEAT_FORCE | FEAT_DRAG>{});
        case FEAT_EQ2: return go(std::integral_constant<int, FEAT_EQ2>{});
        case FEAT_EQ2 | FEAT_FORCE | FEAT_DRAG:
          return go(std::integral_constant<int, FEAT_EQ2 | FEAT_FORCE | FEAT_DRAG>{});
        default: break;
      }
    }
    return by_variant(b->lats[0], [&](auto walls, auto feat) -> int {
      if constexpr (decltype(feat)::value == FEAT_ALL || decltype(feat)::value == FEAT_MOVING) {
        return fail(VANSE_ERR_UNSUPPORTED, "batches take no time-varying phi, nor a scheme variant with solid nodes");
      } else {
        return batch_launch_t<S, T, SH, decltype(walls)::value, decltype(feat)::value>(b, launch, st);
      }
    });
  });
}

}  // namespace

extern "C" {

int vanse_batch_workspace_bytes_ex(vanse_lattice* const* lats, int n, int threads, int rows,
                                   int steps_per_pass, size_t* bytes) {
  if (!bytes) return fail(VANSE_ERR_INVALID_ARG, "bytes is NULL");
  std::vector<int> r, f;
  int tiles;
  size_t eo, to;
  return batch_layout(lats, n, threads, rows, steps_per_pass, &r, &f, &tiles, &eo, &to, bytes);
}

int vanse_batch_workspace_bytes(vanse_lattice* const* lats, int n, int threads, int rows, size_t* bytes) {
  return vanse_batch_workspace_bytes_ex(lats, n, threads, rows, 1, bytes);
}

int vanse_batch_create_ex(vanse_lattice* const* lats, int n, int threads, int rows, int steps_per_pass,
                          void* workspace, size_t bytes, vanse_batch** out) {
  if (!out) return fail(VANSE_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  std::vector<int> r, f;
  int tiles;
  size_t eo, to, need;
  if (int rc = batch_layout(lats, n, threads, rows, steps_per_pass, &r, &f, &tiles, &eo, &to, &need))
    return rc;
  if (!workspace || (((uintptr_t)workspace) & 255)) return fail(VANSE_ERR_WORKSPACE, "batch workspace missing or not 256-byte aligned");
  if (bytes < need) return fail(VANSE_ERR_WORKSPACE, "batch workspace too small: %zu < %zu", bytes, need);
  vanse_batch* b = new (std::nothrow) vanse_batch();
  if (!b) return fail(VANSE_ERR_INVALID_ARG, "out of host memory");
  b->lats.assign(lats, lats + n);
  b->rows = r;
  b->first = f;
  b->threads = threads;
  b->fuse = steps_per_pass;
  b->total_tiles = tiles;
  b->ws = static_cast<char*>(workspace);
  b->entries_off = eo;
  b->tiles_off = to;
  *out = b;
  return VANSE_OK;
}

int vanse_batch_create(vanse_lattice* const* lats, int n, int threads, int rows, void* workspace,
                       size_t bytes, vanse_batch** out) {
  return vanse_batch_create_ex(lats, n, threads, rows, 1, workspace, bytes, out);
}

int vanse_batch_destroy(vanse_batch* b) {
  if (!b) return VANSE_OK;
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->own) (void)hipStreamDestroy(b->own);
  delete b;
  return VANSE_OK;
}

int vanse_batch_set_graph(vanse_batch* b, int steps_per_graph) {
  if (!b) return fail(VANSE_ERR_INVALID_ARG, "batch is NULL");
  // a graph replays an even number of launches (each member's buffers end
  // where they started)
  const int period = 2 * b->fuse;
  if (steps_per_graph < 0 || steps_per_graph % period)
    return fail(VANSE_ERR_INVALID_ARG, "steps per graph must be 0 or a positive multiple of %d (got %d)", period,
                steps_per_graph);
  if (b->graph) {
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  b->graph_steps = steps_per_graph;
  return VANSE_OK;
}

int vanse_batch_tiles(const vanse_batch* b, int* tiles, int* rows) {
  if (!b) return fail(VANSE_ERR_INVALID_ARG, "batch is NULL");
  if (tiles) *tiles = b->total_tiles;
  if (rows) *rows = b->rows.empty() ? 0 : b->rows[0];
  return VANSE_OK;
}

int vanse_batch_step(vanse_batch* b, int64_t nsteps, void* stream) {
  if (!b) return fail(VANSE_ERR_INVALID_ARG, "batch is NULL");
  if (nsteps < 0) return fail(VANSE_ERR_INVALID_ARG, "nsteps must be >= 0");
  for (vanse_lattice* h : b->lats) {
    if (int rc = check_ready(h)) return rc;
    if (!h->state_set) return fail(VANSE_ERR_STATE, "a lattice of the batch has no populations");
    if (!batch_ok(h)) return fail(VANSE_ERR_UNSUPPORTED, "a lattice of the batch uses a variant batches do not take");
  }
  if (nsteps == 0) return VANSE_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the table snapshots each lattice's buffer parity and parameters: upload
  // again if a member changed or was stepped on its own since
  bool stale = !b->table_ready || b->launched > (1LL << 40);
  for (size_t k = 0; !stale && k < b->lats.size(); ++k)
    stale = b->lats[k]->version != b->versions[k] ||
            b->lats[k]->cur != ((b->cur0[k] + (int)(b->launched & 1)) & 1);
  if (stale) {
    if (int rc = batch_upload(b, st)) return rc;
  }
  // launches of `fuse` steps each; with two steps per launch an odd count
  // ends with one step of each member on its own
  const int64_t launches = nsteps / b->fuse;
  const int64_t rem = nsteps % b->fuse;
  const int glaunch = b->graph_steps / b->fuse;  // launches per graph
  int64_t left = launches;
  if (glaunch > 0 && left >= glaunch) {
    if (!b->own) {
      HIP_TRY(hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
      HIP_TRY(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    }
    // graph replays assume an even launch count at their start
    if (b->launched & 1) {
      if (int rc = batch_launch(b, (int)(b->launched & 1), st)) return rc;
      b->launched += 1;
      left -= 1;
    }
    HIP_TRY(hipEventRecord(b->ev_in, st));
    HIP_TRY(hipStreamWaitEvent(b->own, b->ev_in, 0));
    if (!b->graph && left >= glaunch) {
      hipGraph_t graph;
      HIP_TRY(hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal));
      int lrc = VANSE_OK;
      for (int s = 0; s < glaunch && lrc == VANSE_OK; ++s) lrc = batch_launch(b, s, b->own);
      const hipError_t ce = hipStreamEndCapture(b->own, &graph);
      if (lrc != VANSE_OK) {
        if (ce == hipSuccess) (void)hipGraphDestroy(graph);
        return lrc;
      }
      if (ce != hipSuccess) return fail(VANSE_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ce));
      const hipError_t e = hipGraphInstantiate(&b->graph, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return fail(VANSE_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    while (left >= glaunch) {
      HIP_TRY(hipGraphLaunch(b->graph, b->own));
      b->launched += glaunch;
      left -= glaunch;
    }
    HIP_TRY(hipEventRecord(b->ev_out, b->own));
    HIP_TRY(hipStreamWaitEvent(st, b->ev_out, 0));
  }
  for (int64_t s = 0; s < left; ++s) {
    if (int rc = batch_launch(b, (int)(b->launched & 1), st)) return rc;
    b->launched += 1;
  }
  HIP_TRY(hipGetLastError());
  // keep every member handle consistent with the batch
  for (size_t k = 0; k < b->lats.size(); ++k) {
    vanse_lattice* h = b->lats[k];
    h->t += launches * b->fuse;
    h->cur = (h->cur + (int)(launches & 1)) & 1;
  }
  for (size_t k = 0; rem && k < b->lats.size(); ++k)
    if (int rc = vanse_step(b->lats[k], rem, stream)) return rc;
  return VANSE_OK;
}

int vanse_batch_residual(vanse_batch* b, double* out, void* stream) {
  if (!b) return fail(VANSE_ERR_INVALID_ARG, "batch is NULL");
  if (!out) return fail(VANSE_ERR_INVALID_ARG, "out is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t n = b->lats.size();
  double* recs = reinterpret_cast<double*>(
      b->ws + align256(b->tiles_off + (size_t)b->total_tiles * sizeof(int2)));
  std::vector<char> had(n);
  // each member's read-out and reduction as vanse_residual, the final record
  // into the batch's record array; one copy and one synchronization for all
  for (size_t k = 0; k < n; ++k) {
    vanse_lattice* h = b->lats[k];
    had[k] = h->uprev_valid;
    if (int rc = moments(h, nullptr, nullptr, nullptr, nullptr, true, stream, true)) return rc;
    const long long nblk = (long long)((h->d.nx + 255) / 256) * h->d.ny;
    if (int rc = reduce_blocks((const double*)(h->ws + h->L.partials), nblk, (double*)(h->ws + h->L.partials2),
                               recs + k * NOBS, st))
      return rc;
  }
  std::vector<double> rec(n * NOBS);
  HIP_TRY(hipMemcpyAsync(rec.data(), recs, rec.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double bad = 0.0;
  for (size_t k = 0; k < n; ++k) {
    b->lats[k]->uprev_valid = true;
    out[3 * k + 0] = had[k] ? rec[k * NOBS + 4] : -1.0;
    out[3 * k + 1] = rec[k * NOBS + 1];
    out[3 * k + 2] = rec[k * NOBS + 3];
    bad += rec[k * NOBS + 3];
  }
  if (bad > 0) return fail(VANSE_ERR_DIVERGED, "%.0f nodes of the batch hold non-finite values", bad);
  return VANSE_OK;
}

const char* vanse_error_string(int code) {
  switch (code) {
    case VANSE_OK: return "ok";
    case VANSE_ERR_INVALID_ARG: return "invalid argument";
    case VANSE_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case VANSE_ERR_HIP: return "HIP runtime error";
    case VANSE_ERR_STATE: return "lattice not ready";
    case VANSE_ERR_DIVERGED: return "non-finite values observed";
    case VANSE_ERR_UNSUPPORTED: return "unsupported variant";
  }
  return "unknown error";
}

const char* vanse_last_error(void) { return g_err; }

}  // extern "C"
