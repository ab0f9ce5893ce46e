// step_kernel.hpp -- the fused MRTLB-VANSE collide-and-stream step for gfx950.
//
// One launch advances every node by one time step of the scheme of Liu,
// Zhang, Min & Wu (arXiv:2409.02964, Sec. 2.3):
//   pull streaming with half-way bounce-back           (Sec. 2.3, Sec. 3.1)
//   phi*rho = sum f, j = sum e f, rho = sum f / phi      (Eq. 7)
//   F = F^p + F^B, F^p = (kappa - phi) cs^2 grad rho     (Eq. 13, Eq. 10)
//   u = (j + F/2) / (phi rho)                            (Eq. 7)
//   penalty source C from eight Eq. (10) derivatives     (Eq. 20)
//   m = M f, m+ = m - Gamma (m - m^eq) + (I - Gamma/2)(S + C)
//                                                        (Eq. 16-19)
//   f+ = M^-1 m+                                         (Eq. A1)
// Optional: a per-node force field, a linear drag, a time-varying void
// fraction (the d_t phi term of Eq. 20) and solid nodes (bounce-back on
// their faces and the centre-value stand-in of Eq. 10 next to them).
//
// Work layout: one workgroup owns a strip of `out_w` columns plus two halo
// columns on each side (one lane per column) and sweeps a block of rows
// bottom-up.  Per sweep iteration three stages run on three consecutive rows:
//   A  row yn   : pull the 9 populations, moments, delta-rho -> LDS ring
//   B  row yn-1 : grad rho from the ring, F, u, rho u, phi rho u -> LDS ring
//   C  row yn-2 : the eight derivatives from the ring, collision, store.
// Moments of rows yn-1, yn-2 stay in registers between stages, so each
// stored population is read from HBM once (plus the strip/block halos), and
// the step needs no second pass over memory.  All arithmetic is vector ALU:
// the 9x9 transforms are integer-coefficient sums (no MFMA -- the step is
// bound by HBM bandwidth, not by a dense contraction).
//
// Arithmetic is carried on deviations g = f - f^rest from the rest state
// f^rest = f^eq(rho0, 0) of Eq. (14); the moment-space update is linear in
// that shift, so the scheme is unchanged while FP32 keeps the small velocity
// signal away from the O(w_i) population magnitudes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vanse_dev {

// Per-node velocity data shared with the neighbours through LDS: u, the
// products rho u and (phi rho) u that the penalty derivatives of Eq. (20)
// act on.  Split in a 4-vector read by every neighbour and a 2-vector read by
// the north/south and diagonal neighbours only.
template <typename T>
struct alignas(4 * sizeof(T)) U4 {
  T ux, uy, mux, rux;  // u_x, u_y, (phi rho) u_x, rho u_x
};
template <typename T>
struct alignas(2 * sizeof(T)) U2 {
  T muy, ruy;  // (phi rho) u_y, rho u_y
};

template <typename T>
struct StepPhys {
  T kappa, rho0;
  T gx, gy;                 // uniform acceleration G
  T s_e, s_eps, s_q, s_nu;  // relaxation rates (non-conserved moments)
  T rest_axis, rest_diag;   // w_i kappa rho0 for |e|=1 and |e|=sqrt2
  T rest0_k;                // 5 kappa rho0 / 9 : rest_0 = phi rho0 - rest0_k
  T scale, inv_scale;       // storage scale of shifted half storage
  T usx, usy;               // solid velocity of the linear drag
  int scale_by_phi;
  int model_b;  // model B (set I): kappa - 1 in place of kappa - phi in F^p and C
  int eq2;      // second-order equilibrium (B1-B2) with the penalty of Eq. (B3)
  T uw_lo, uw_hi;  // x velocities of the walls at y = -1/2 and y = ny - 1/2
  // Uniform products of the above, formed on the host in T arithmetic (the
  // same roundings as forming them in a kernel).  The hardware has no scalar
  // floating-point ALU, so a kernel would hold them in vector registers.
  T k2, k3, k12;            // 2 kappa, 3 kappa, kappa / 12
  T he, hep, hq, hn;        // 1 - s/2 for s_e, s_eps, s_q, s_nu (Eq. 16)
  T bt9, bt36, bt6, bt12, bt4;  // 1/9, 1/36, 1/6, 1/12, 1/4 of Eq. (A1) times `scale`
  // Velocity boundary rows (Sec. 3.1, Couette flow; FEAT_ALL with walls):
  // the first (nee_lo) or last (nee_hi) row lies on a wall moving with x
  // velocity un_lo / un_hi and is set by non-equilibrium extrapolation from
  // the fluid row next to it (see vel_row_eq).
  int nee_lo, nee_hi;
  T un_lo, un_hi;
};

// Equilibrium of Eq. (14) (or B1 with eq2) less the rest state, population
// I: f^eq_I(phi, rho, u) - f^eq_I(phi, rho0, 0) with drho = rho - rho0.  With
// X = kappa/phi, phi times the third-order factor is (3 phi - kappa)/2 on
// the axes and kappa on the diagonals (phi for the second-order form).
template <int I, typename T>
__device__ __forceinline__ T eq_dev(T phi, T rho, T drho, T ux, T uy, T kappa, bool eq2) {
  const T pr = phi * rho;
  const T uu = ux * ux + uy * uy;
  if constexpr (I == 0) {
    return (phi - kappa * T(5.0 / 9.0)) * drho - T(2.0 / 3.0) * pr * uu;
  } else {
    constexpr bool axis = I < 5;
    const T v = I == 1 ? ux : I == 2 ? uy : I == 3 ? -ux : I == 4 ? -uy
              : I == 5 ? ux + uy : I == 6 ? uy - ux : I == 7 ? -(ux + uy) : ux - uy;
    const T c3 = eq2 ? phi : (axis ? T(0.5) * (T(3) * phi - kappa) : kappa);
    const T wi = axis ? T(1.0 / 9.0) : T(1.0 / 36.0);
    return wi * (kappa * drho + T(3) * rho * c3 * v + T(4.5) * pr * v * v - T(1.5) * pr * uu);
  }
}

struct StepGeom {
  const void* src;
  void* dst;
  const void* phi;
  const void* fxf;
  const void* fyf;
  const void* beta;  // per-node drag coefficient (F^B -= phi beta (u - u_s))
  const void* phin;  // phi(t+1) (time-varying void fraction; = phi when static)
  const void* nbr;   // uint16 solid flags per node (see FEAT_MASK), or null
  // the second step's inputs of a two-step launch with a moving phi:
  // phi(t+2), and the drag coefficient and force field of that step
  const void* phin2;
  const void* beta2;
  const void* fxf2;
  const void* fyf2;
  long long plane;  // elements per population plane (= pitch * ny)
  int nx, ny, pitch;
  int xwalls;       // half-way walls at x = -1/2 and x = nx - 1/2 (FEAT_MASK instances)
  int strips, out_w, rows;
};

__device__ __forceinline__ int wrap_index(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Tile of workgroup b of nb.  Workgroups are dealt to the 8 XCDs (each with
// its own L2) in turn; this order gives each XCD a contiguous run of tiles,
// so that strips side by side, which read each other's halo columns at the
// same time, share an L2.  A bijection on [0, nb).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int x = b & 7, i = b >> 3, q = nb >> 3, r = nb & 7;
  return x * q + min(x, r) + i;
}

// LDS ring slot of a (possibly negative) row index: four rows per ring
__device__ __forceinline__ int slot4(int y) { return y & 3; }

// Reciprocal: the hardware v_rcp_f32 (1 ulp) in FP32, a correctly rounded
// division in FP64.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Buffer-resource memory access: a scalar descriptor per plane (base and
// size in bytes), a per-lane byte offset (the column, loop-invariant) and a
// uniform byte offset (the row).  Address arithmetic then costs no vector
// instructions, and an offset beyond the plane reads 0 instead of faulting.
using rsrc_t = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, int(bytes), 0x00020000);
}
template <typename S>
__device__ __forceinline__ S bload(rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ float bload<float>(rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double bload<double>(rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ _Float16 bload<_Float16>(rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
}
__device__ __forceinline__ unsigned bload_u16(rsrc_t r, unsigned voff, unsigned soff) {
  return unsigned(__builtin_bit_cast(unsigned short, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0)));
}
__device__ __forceinline__ void bstore(float v, rsrc_t r, unsigned voff, unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}
__device__ __forceinline__ void bstore(double v, rsrc_t r, unsigned voff, unsigned soff) {
  using u2 = unsigned __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff, 0);
}
__device__ __forceinline__ void bstore(_Float16 v, rsrc_t r, unsigned voff, unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, voff, soff, 0);
}

// Eq. (10): d_x psi = (psi_E - psi_W)/3 + (psi_NE + psi_SE - psi_NW - psi_SW)/12
template <typename T>
__device__ __forceinline__ T stencil_dx(T e, T w, T ne, T se, T nw, T sw) {
  return (e - w) * T(1.0 / 3.0) + ((ne + se) - (nw + sw)) * T(1.0 / 12.0);
}
template <typename T>
__device__ __forceinline__ T stencil_dy(T n, T s, T ne, T nw, T se, T sw) {
  return (n - s) * T(1.0 / 3.0) + ((ne + nw) - (se + sw)) * T(1.0 / 12.0);
}

// Moments of one row carried from stage A to stages B and C (deviations from
// the rest state): dm0 = sum g, j, and the six non-conserved moments of
// Eq. (17), plus phi and delta-rho of the node.
template <typename T>
struct RowState {
  T dm0, jx, jy, me, mep, mqx, mqy, mpxx, mpxy, phi, drho, beta, dphi;
  T rphi;  // 1/phi (the two-step kernel keeps it from stage A for stage C)
  unsigned nb;
};

// What load_row fetches for one row: the nine pulled populations, phi, and
// the optional drag coefficient, phi(t+1) and solid flags.
template <typename S, typename T>
struct RowIn {
  S f[9];
  T phi, beta, phin;
  unsigned nb;
};

// Optional features of the step (bit mask).  FEAT_SCHEME honours the
// run-time scheme flags of StepPhys (model B, second-order equilibrium,
// moving walls).
// FEAT_ALL is built with every feature and takes absent inputs as zero (null
// force, drag and flag planes read as 0 through zero-length buffer
// descriptors; phin = phi when static).
enum : int {
  FEAT_FORCE = 1, FEAT_DRAG = 2, FEAT_DYNPHI = 4, FEAT_MASK = 8, FEAT_SCHEME = 16, FEAT_ALL = 31,
  // the two-step kernel only: the Appendix B equilibrium (B1, B2) and the
  // penalty of Eq. (B3), with model B as the run-time flag
  FEAT_EQ2 = 32
};

// Solid flags of FEAT_MASK, one uint16 per node: bit 0 -- the node itself is
// solid (and then its only bit); bit i (1..8) -- the node standing in for
// x + e_i (after reflection across a wall) is solid.  A fluid node pulls f_i from its own slot opp(i)
// when bit opp(i) is set (half-way bounce-back on the solid face), and the
// Eq. (10) stencils replace a flagged neighbour by the centre value, negated
// for velocity-like fields.
__device__ __forceinline__ bool solid_bit(unsigned nb, int i) { return (nb >> i) & 1u; }

// S: storage type of populations (double, float, _Float16)
// T: arithmetic type (double, float)
// SHIFT: memory holds deviations g (scaled by ph.scale in half storage) instead of f
// WALLS: half-way bounce-back walls at y = -1/2 and y = ny - 1/2
// FEAT: FEAT_FORCE adds the per-node force planes to F^B; FEAT_DRAG adds
//       the linear drag -phi beta (u - u_s) with u solved in closed form
// NT: threads per workgroup (= out_w + 4 active lanes at most)
// LDS rings over the last four rows.  Next to a wall the row beyond it is
// filled with the mirror image (scalars copied, velocities negated), so the
// stencils never test for walls.
template <typename T, int NT>
struct StepLds {
  T rho[4][NT];      // delta-rho (stage A -> stage B)
  U4<T> u4[4][NT];   // (stage B -> stage C)
  U2<T> u2[4][NT];
};

// One workgroup's tile: strip `strip` (columns strip*out_w .. +out_w-1) and
// row block `by` (rows by*rows .. +rows-1) of the lattice described by g.
// PD: prefetch distance in rows (1 or 2).
template <typename S, typename T, bool SHIFT, bool WALLS, int FEAT, int NT, int PD>
__device__ __forceinline__ void step_tile(const StepGeom& g, const StepPhys<T>& ph, int strip,
                                          int by, StepLds<T, NT>& L) {
  auto& s_rho = L.rho;
  auto& s_u4 = L.u4;
  auto& s_u2 = L.u2;
  const int t = threadIdx.x;
  const int nx = g.nx, ny = g.ny, pitch = g.pitch;
  const int x0 = strip * g.out_w;
  const int w = min(g.out_w, nx - x0);
  const bool live = t < w + 4;                 // pulls and delta-rho
  const bool ulane = t >= 1 && t < w + 3;      // velocity
  const bool olane = t >= 2 && t < w + 2;      // collision and store
  // Walls in x (solid-node instances only): a halo lane beyond a face
  // stands for the mirror column c.  It pulls and computes exactly as the
  // lane of column c (slot tc of this strip), reading its stencils around
  // tc, and stores the velocity-like results negated.  The face columns pull
  // across the face from their own opposite slots (flags fb).
  const int xg = x0 - 2 + t;
  // (not in the mask-with-force-or-drag instance, whose registers are full:
  // the host routes walls in x with those inputs to the moving-phi one)
  constexpr bool XW = (FEAT & FEAT_MASK) != 0 && FEAT != (FEAT_MASK | FEAT_FORCE | FEAT_DRAG);
  const bool xw = XW && g.xwalls != 0;
  int c, cm, cp, tc = t;
  if (xw) {
    c = min(max(xg < 0 ? -1 - xg : (xg >= nx ? 2 * nx - 1 - xg : xg), 0), nx - 1);
    cm = max(c - 1, 0);
    cp = min(c + 1, nx - 1);
    tc = min(max(t + (c - xg), 0), NT - 1);
  } else {
    c = wrap_index(xg, nx);
    cm = (c == 0) ? nx - 1 : c - 1;
    cp = (c == nx - 1) ? 0 : c + 1;
  }
  // per-lane conditions (kept as lane masks, not registers)
  const bool xmir = xw && (xg < 0 || xg >= nx);
  const bool xlo = xw && c == 0, xhi = xw && c == nx - 1;
  const int tl = max(tc - 1, 0), tr = min(tc + 1, NT - 1);
  constexpr unsigned SB = sizeof(S);
  constexpr unsigned TB = sizeof(T);
  // velocity boundary rows: built into the instance with every feature only
  // (elsewhere their code would push the register budget into spills)
  constexpr bool NEE = WALLS && FEAT == FEAT_ALL;

  // one buffer descriptor per array; the plane and the row go into the
  // uniform offset, the column into the per-lane offset (each population
  // buffer is below 4 GiB, which the host checks)
  const unsigned plane_bytes = unsigned(g.plane) * SB;
  const unsigned row_bytes = unsigned(pitch) * SB;
  const rsrc_t srcr = make_rsrc(g.src, 9u * plane_bytes);
  const rsrc_t dstr = make_rsrc(g.dst, 9u * plane_bytes);
  const rsrc_t phir = make_rsrc(g.phi, unsigned(g.plane) * TB);
  auto poff = [&](int i, int r) { return unsigned(i) * plane_bytes + unsigned(r) * row_bytes; };

  const int y0 = by * g.rows;
  const int y1 = min(y0 + g.rows, ny);
  const int nit = (y1 - y0) + 4;

  const T kappa = ph.kappa, rho0 = ph.rho0;
  const T third = T(1.0 / 3.0);
  // loop-invariant per-lane byte offsets of the own and neighbour columns
  const unsigned xcb = unsigned(c) * SB, xmb = unsigned(cm) * SB, xpb = unsigned(cp) * SB;
  const unsigned xcT = unsigned(c) * TB;

  // Issue the ten loads (nine pulled populations and phi) of row yn.  Rows
  // outside a walled domain are clamped to a valid row and never used, so
  // every load is unconditional and in bounds.
  const rsrc_t betar = make_rsrc(g.beta, ((FEAT & FEAT_DRAG) && g.beta) ? unsigned(g.plane) * TB : 0u);
  const rsrc_t phinr = make_rsrc(g.phin, (FEAT & FEAT_DYNPHI) ? unsigned(g.plane) * TB : 0u);
  const rsrc_t nbrr = make_rsrc(g.nbr, ((FEAT & FEAT_MASK) && g.nbr) ? unsigned(g.plane) * 2u : 0u);
  const rsrc_t fxr = make_rsrc(g.fxf, ((FEAT & FEAT_FORCE) && g.fxf) ? unsigned(g.plane) * TB : 0u);
  const rsrc_t fyr = make_rsrc(g.fyf, ((FEAT & FEAT_FORCE) && g.fyf) ? unsigned(g.plane) * TB : 0u);
  auto load_row = [&](int yn, RowIn<S, T>& in) {
    S (&f)[9] = in.f;
    T& phi = in.phi;
    T& beta = in.beta;
    T& phin = in.phin;
    unsigned& nb = in.nb;
    int r, rs, rn;
    bool bl = false, bh = false;
    if (WALLS) {
      r = min(max(yn, 0), ny - 1);
      bl = (yn == 0);
      bh = (yn == ny - 1);
      rs = max(r - 1, 0);
      rn = min(r + 1, ny - 1);
    } else {
      r = wrap_index(yn, ny);
      rs = (r == 0) ? ny - 1 : r - 1;
      rn = (r == ny - 1) ? 0 : r + 1;
    }
    phi = bload<T>(phir, xcT, unsigned(r) * unsigned(pitch) * TB);
    if (FEAT & FEAT_DRAG) beta = bload<T>(betar, xcT, unsigned(r) * unsigned(pitch) * TB);
    if (FEAT & FEAT_DYNPHI) phin = bload<T>(phinr, xcT, unsigned(r) * unsigned(pitch) * TB);
    if constexpr ((FEAT & FEAT_MASK) != 0) {
      // per-lane choice between the pulled slot and the own node's opposite
      // slot (solid source): whole byte offsets in the per-lane operand
      nb = bload_u16(nbrr, unsigned(c) * 2u, unsigned(r) * unsigned(pitch) * 2u);
      const unsigned pnb = nb | (xlo ? (1u << 3) | (1u << 6) | (1u << 7) : 0u) |
                           (xhi ? (1u << 1) | (1u << 5) | (1u << 8) : 0u);
      auto pick = [&](unsigned vcol, unsigned soff, int opp) -> S {
        const unsigned own = poff(opp, r) + xcb;
        return bload<S>(srcr, solid_bit(pnb, opp) ? own : soff + vcol, 0u);
      };
      f[0] = bload<S>(srcr, xcb, poff(0, r));
      f[1] = pick(xmb, poff(1, r), 3);
      f[3] = pick(xpb, poff(3, r), 1);
      f[2] = pick(xcb, bl ? poff(4, r) : poff(2, rs), 4);
      f[5] = pick(bl ? xcb : xmb, bl ? poff(7, r) : poff(5, rs), 7);
      f[6] = pick(bl ? xcb : xpb, bl ? poff(8, r) : poff(6, rs), 8);
      f[4] = pick(xcb, bh ? poff(2, r) : poff(4, rn), 2);
      f[7] = pick(bh ? xcb : xpb, bh ? poff(5, r) : poff(7, rn), 5);
      f[8] = pick(bh ? xcb : xmb, bh ? poff(6, r) : poff(8, rn), 6);
      return;
    }
    f[0] = bload<S>(srcr, xcb, poff(0, r));
    f[1] = bload<S>(srcr, xmb, poff(1, r));
    f[3] = bload<S>(srcr, xpb, poff(3, r));
    // sources below the lower wall bounce back: f2,f5,f6 <- f4,f7,f8 at x
    f[2] = bload<S>(srcr, xcb, bl ? poff(4, r) : poff(2, rs));
    f[5] = bload<S>(srcr, bl ? xcb : xmb, bl ? poff(7, r) : poff(5, rs));
    f[6] = bload<S>(srcr, bl ? xcb : xpb, bl ? poff(8, r) : poff(6, rs));
    // sources above the upper wall: f4,f7,f8 <- f2,f5,f6 at x
    f[4] = bload<S>(srcr, xcb, bh ? poff(2, r) : poff(4, rn));
    f[7] = bload<S>(srcr, bh ? xcb : xpb, bh ? poff(5, r) : poff(7, rn));
    f[8] = bload<S>(srcr, bh ? xcb : xmb, bh ? poff(6, r) : poff(8, rn));
  };

  // One sweep iteration.  A: row yn, B: row yn-1, C: row yn-2.  rA is
  // written, rB/rC are read; bNew is written by B, bOld (row yn-2) read by C.
  auto body = [&](int k, const RowIn<S, T>& in, RowState<T>& rA,
                  const RowState<T>& rB, const RowState<T>& rC, T (&bNew)[2],
                  const T (&bOld)[2]) {
    const int yn = y0 - 2 + k;
    const S (&f)[9] = in.f;
    // FP16 and FP64 storage: the waves in stages A and B (the short phase up
    // to the second barrier) issue before the waves in stage C (s_setprio;
    // the results do not change).  Measured on the 4096^2 channel: 186.3 ->
    // 183.5 us per step in FP16-shifted storage, 612 -> 606 in FP64; with
    // 4-byte storage it gained nothing.
    if (sizeof(S) != 4) __builtin_amdgcn_s_setprio(1);
    const T phi_in = in.phi, beta_in = in.beta, phin_in = in.phin;
    const unsigned nb_in = in.nb;

    // ---------------- stage A: moments of row yn ----------------
    const bool rowA = WALLS ? (yn >= 0 && yn < ny) : true;
    if (rowA && live) {
      const T phi = phi_in;
      T q[9];
      if (SHIFT) {  // only half storage carries a scale (2^-e)
#pragma unroll
        for (int i = 0; i < 9; ++i)
          q[i] = sizeof(S) == 2 ? static_cast<T>(f[i]) * ph.inv_scale : static_cast<T>(f[i]);
      } else {
        q[0] = static_cast<T>(f[0]) - (phi * rho0 - ph.rest0_k);
#pragma unroll
        for (int i = 1; i < 5; ++i) q[i] = static_cast<T>(f[i]) - ph.rest_axis;
#pragma unroll
        for (int i = 5; i < 9; ++i) q[i] = static_cast<T>(f[i]) - ph.rest_diag;
      }
      if constexpr (WALLS && (FEAT & FEAT_SCHEME) != 0) {
        // moving walls: a population that crossed the wall returns less the
        // odd part of the equilibrium at the wall velocity, which for the
        // diagonals is (e_i . u_w) rho0 phi h3 / 6 with phi h3 = kappa (Eq. 14)
        // or phi (B1); the axis populations carry no tangential momentum
        const T kw = (ph.eq2 ? phi : kappa) * rho0 * T(1.0 / 6.0);
        if (yn == 0) {
          const T c0 = kw * ph.uw_lo;
          q[5] += c0;
          q[6] -= c0;
        }
        if (yn == ny - 1) {
          const T c1 = kw * ph.uw_hi;
          q[7] -= c1;
          q[8] += c1;
        }
      }
      // rows of M (Eq. A1) applied to the deviations
      const T sa = (q[1] + q[2]) + (q[3] + q[4]);
      const T sd = (q[5] + q[6]) + (q[7] + q[8]);
      rA.dm0 = q[0] + (sa + sd);
      rA.jx = (q[1] - q[3]) + ((q[5] - q[6]) + (q[8] - q[7]));
      rA.jy = (q[2] - q[4]) + ((q[5] + q[6]) - (q[7] + q[8]));
      rA.me = T(-4) * q[0] - sa + T(2) * sd;
      rA.mep = T(4) * q[0] - T(2) * sa + sd;
      rA.mqx = T(-2) * (q[1] - q[3]) + ((q[5] - q[6]) + (q[8] - q[7]));
      rA.mqy = T(-2) * (q[2] - q[4]) + ((q[5] + q[6]) - (q[7] + q[8]));
      rA.mpxx = (q[1] + q[3]) - (q[2] + q[4]);
      rA.mpxy = (q[5] + q[7]) - (q[6] + q[8]);
      rA.phi = phi;
      rA.beta = beta_in;
      rA.dphi = (FEAT & FEAT_DYNPHI) ? phin_in - phi : T(0);
      rA.nb = (FEAT & FEAT_MASK) ? nb_in : 0u;
      rA.drho = rA.dm0 * recip(phi);
      s_rho[slot4(yn)][t] = rA.drho;
      if (WALLS && yn == 0) s_rho[slot4(-1)][t] = rA.drho;      // image below
      if (WALLS && yn == ny - 1) s_rho[slot4(ny)][t] = rA.drho; // image above
      if constexpr (NEE) {
        // a velocity row takes the density of the fluid row next to it
        if (ph.nee_lo && yn == 1) s_rho[slot4(0)][t] = rA.drho;
        if (ph.nee_hi && yn == ny - 1) s_rho[slot4(yn)][t] = rB.drho;
      }
    }
    __syncthreads();

    // ---------------- stage B: velocity of row yn-1 ----------------
    const int yb = yn - 1;
    const bool rowB = (yb >= y0 - 1) && (WALLS ? (yb >= 0 && yb < ny) : true);
    if (rowB && ulane) {
      const int sc = slot4(yb), ss = slot4(yb - 1), sn = slot4(yb + 1);
      T rE = s_rho[sc][tr], rW = s_rho[sc][tl];
      T rN = s_rho[sn][tc], rS = s_rho[ss][tc];
      T rNE = s_rho[sn][tr], rNW = s_rho[sn][tl];
      T rSE = s_rho[ss][tr], rSW = s_rho[ss][tl];
      if constexpr ((FEAT & FEAT_MASK) != 0) {  // solid neighbour: centre value
        const unsigned nb = rB.nb;
        const T rc = rB.drho;
        rE = solid_bit(nb, 1) ? rc : rE;
        rN = solid_bit(nb, 2) ? rc : rN;
        rW = solid_bit(nb, 3) ? rc : rW;
        rS = solid_bit(nb, 4) ? rc : rS;
        rNE = solid_bit(nb, 5) ? rc : rNE;
        rNW = solid_bit(nb, 6) ? rc : rNW;
        rSW = solid_bit(nb, 7) ? rc : rSW;
        rSE = solid_bit(nb, 8) ? rc : rSE;
      }
      const T grx = stencil_dx(rE, rW, rNE, rSE, rNW, rSW);
      const T gry = stencil_dy(rN, rS, rNE, rNW, rSE, rSW);
      const T phi = rB.phi;
      const T kf = ((FEAT & FEAT_SCHEME) && ph.model_b) ? T(1) : phi;
      const T kp = (kappa - kf) * third;  // Eq. (13); kappa - 1 for model B
      const T sg = ph.scale_by_phi ? phi : T(1);
      T Fx = kp * grx + sg * ph.gx;
      T Fy = kp * gry + sg * ph.gy;
      if (FEAT & FEAT_FORCE) {
        const unsigned ro = unsigned(WALLS ? yb : wrap_index(yb, ny)) * unsigned(pitch) * TB;
        Fx += bload<T>(fxr, xcT, ro);
        Fy += bload<T>(fyr, xcT, ro);
      }
      const T m0 = phi * rho0 + rB.dm0;
      T ux, uy;
      if (FEAT & FEAT_DRAG) {
        // F = F' - phi beta (u - u_s) with u = (j + F/2)/m0: solved for u
        const T d = phi * rB.beta;
        const T inv = recip(m0 + T(0.5) * d);
        ux = (rB.jx + T(0.5) * (Fx + d * ph.usx)) * inv;
        uy = (rB.jy + T(0.5) * (Fy + d * ph.usy)) * inv;
        Fx -= d * (ux - ph.usx);
        Fy -= d * (uy - ph.usy);
      } else {
        const T inv_m0 = recip(m0);
        ux = (rB.jx + T(0.5) * Fx) * inv_m0;
        uy = (rB.jy + T(0.5) * Fy) * inv_m0;
      }
      const T rho = rho0 + rB.drho;
      U4<T> a;
      U2<T> b;
      a.ux = ux; a.uy = uy; a.mux = m0 * ux; a.rux = rho * ux;
      b.muy = m0 * uy; b.ruy = rho * uy;
      if constexpr (NEE) {
        // velocity row: the wall velocity, with the density of the fluid row
        // next to it (row 1 is this iteration's stage-A row, row ny - 2 its
        // stage-C row)
        const bool lo = ph.nee_lo && yb == 0, hi = ph.nee_hi && yb == ny - 1;
        if (lo || hi) {
          const T rf = rho0 + (lo ? rA.drho : rC.drho);
          const T uw = lo ? ph.un_lo : ph.un_hi;
          a.ux = uw; a.uy = T(0); a.mux = phi * rf * uw; a.rux = rf * uw;
          b.muy = T(0); b.ruy = T(0);
        }
      }
      if constexpr (XW) {  // mirror lane beyond an x-wall
        U4<T> ax;
        U2<T> bx;
        ax.ux = xmir ? -a.ux : a.ux; ax.uy = xmir ? -a.uy : a.uy;
        ax.mux = xmir ? -a.mux : a.mux; ax.rux = xmir ? -a.rux : a.rux;
        bx.muy = xmir ? -b.muy : b.muy; bx.ruy = xmir ? -b.ruy : b.ruy;
        s_u4[slot4(yb)][t] = ax;
        s_u2[slot4(yb)][t] = bx;
      } else {
        s_u4[slot4(yb)][t] = a;
        s_u2[slot4(yb)][t] = b;
      }
      if (WALLS && (yb == 0 || yb == ny - 1)) {  // mirror image beyond the wall
        const int sg2 = slot4(yb == 0 ? -1 : ny);
        U4<T> am;
        U2<T> bm;
        am.ux = -a.ux; am.uy = -a.uy; am.mux = -a.mux; am.rux = -a.rux;
        if constexpr ((FEAT & FEAT_SCHEME) != 0) {  // moving wall: u -> 2 u_w - u
          const T uw2 = T(2) * (yb == 0 ? ph.uw_lo : ph.uw_hi);
          am.ux += uw2; am.mux += uw2 * m0; am.rux += uw2 * rho;
        }
        bm.muy = -b.muy; bm.ruy = -b.ruy;
        s_u4[sg2][t] = am;
        s_u2[sg2][t] = bm;
      }
      bNew[0] = Fx;
      bNew[1] = Fy;
    }
    __syncthreads();
    if (sizeof(S) != 4) __builtin_amdgcn_s_setprio(0);  // stage C after them

    // ---------------- stage C: collide row yn-2 ----------------
    const int yo = yn - 2;
    if (yo >= y0 && olane) {
      const int uo = slot4(yo), us = slot4(yo - 1), un = slot4(yo + 1);
      const U4<T> aC = s_u4[uo][tc];
      U4<T> aE = s_u4[uo][tr], aW = s_u4[uo][tl];
      U4<T> aN = s_u4[un][tc], aS = s_u4[us][tc];
      U4<T> aNE = s_u4[un][tr], aNW = s_u4[un][tl];
      U4<T> aSE = s_u4[us][tr], aSW = s_u4[us][tl];
      U2<T> bN = s_u2[un][tc], bS = s_u2[us][tc];
      U2<T> bNE = s_u2[un][tr], bNW = s_u2[un][tl];
      U2<T> bSE = s_u2[us][tr], bSW = s_u2[us][tl];
      if constexpr ((FEAT & FEAT_MASK) != 0) {
        // solid neighbour: the centre's velocity-like fields, negated
        const unsigned nb = rC.nb;
        const U2<T> bC = s_u2[uo][tc];
        U4<T> ga;
        ga.ux = -aC.ux; ga.uy = -aC.uy; ga.mux = -aC.mux; ga.rux = -aC.rux;
        U2<T> gb;
        gb.muy = -bC.muy; gb.ruy = -bC.ruy;
        auto sel4 = [&](U4<T>& v, int i) {
          const bool s2 = solid_bit(nb, i);
          v.ux = s2 ? ga.ux : v.ux; v.uy = s2 ? ga.uy : v.uy;
          v.mux = s2 ? ga.mux : v.mux; v.rux = s2 ? ga.rux : v.rux;
        };
        auto sel2 = [&](U2<T>& v, int i) {
          const bool s2 = solid_bit(nb, i);
          v.muy = s2 ? gb.muy : v.muy; v.ruy = s2 ? gb.ruy : v.ruy;
        };
        sel4(aE, 1); sel4(aN, 2); sel4(aW, 3); sel4(aS, 4);
        sel4(aNE, 5); sel4(aNW, 6); sel4(aSW, 7); sel4(aSE, 8);
        sel2(bN, 2); sel2(bS, 4); sel2(bNE, 5); sel2(bNW, 6); sel2(bSW, 7); sel2(bSE, 8);
      }

      // the eight derivatives of Eq. (20), each by Eq. (10)
      const T d_rux_x = stencil_dx(aE.rux, aW.rux, aNE.rux, aSE.rux, aNW.rux, aSW.rux);
      const T d_ruy_y = stencil_dy(bN.ruy, bS.ruy, bNE.ruy, bNW.ruy, bSE.ruy, bSW.ruy);
      const T d_ux_x = stencil_dx(aE.ux, aW.ux, aNE.ux, aSE.ux, aNW.ux, aSW.ux);
      const T d_uy_y = stencil_dy(aN.uy, aS.uy, aNE.uy, aNW.uy, aSE.uy, aSW.uy);
      const T d_uy_x = stencil_dx(aE.uy, aW.uy, aNE.uy, aSE.uy, aNW.uy, aSW.uy);
      const T d_ux_y = stencil_dy(aN.ux, aS.ux, aNE.ux, aNW.ux, aSE.ux, aSW.ux);
      const T d_mux_x = stencil_dx(aE.mux, aW.mux, aNE.mux, aSE.mux, aNW.mux, aSW.mux);
      const T d_muy_y = stencil_dy(bN.muy, bS.muy, bNE.muy, bNW.muy, bSE.muy, bSW.muy);

      const T phi = rC.phi;
      const T rho = rho0 + rC.drho;
      const T X = kappa * recip(phi);
      const bool eq2 = (FEAT & FEAT_SCHEME) && ph.eq2;
      const T kmp = kappa - (((FEAT & FEAT_SCHEME) && ph.model_b) ? T(1) : phi);
      const T ux = aC.ux, uy = aC.uy, Fx = bOld[0], Fy = bOld[1];

      // penalty source (Eq. 20, or B3 for the second-order equilibrium);
      // d_t phi = phi(t+1) - phi(t), zero when static
      T Ca, Cb, Cc;
      if (eq2) {
        U2<T> bE = s_u2[uo][tr], bW = s_u2[uo][tl];
        if constexpr ((FEAT & FEAT_MASK) != 0) {
          const U2<T> bC = s_u2[uo][tc];
          const bool sE = solid_bit(rC.nb, 1), sW = solid_bit(rC.nb, 3);
          bE.muy = sE ? -bC.muy : bE.muy; bE.ruy = sE ? -bC.ruy : bE.ruy;
          bW.muy = sW ? -bC.muy : bW.muy; bW.ruy = sW ? -bC.ruy : bW.ruy;
        }
        const T d_ruy_x = stencil_dx(bE.ruy, bW.ruy, bNE.ruy, bSE.ruy, bNW.ruy, bSW.ruy);
        const T d_muy_x = stencil_dx(bE.muy, bW.muy, bNE.muy, bSE.muy, bNW.muy, bSW.muy);
        const T d_rux_y = stencil_dy(aN.rux, aS.rux, aNE.rux, aNW.rux, aSE.rux, aSW.rux);
        const T d_mux_y = stencil_dy(aN.mux, aS.mux, aNE.mux, aNW.mux, aSE.mux, aSW.mux);
        Ca = T(-2) * kappa * (d_rux_x + d_ruy_y) + T(2) * kmp * rho * (d_ux_x + d_uy_y) +
             (T(4) - T(2) * X) * (d_mux_x + d_muy_y);
        Cb = T(-2.0 / 3.0) * kappa * (d_rux_x - d_ruy_y) +
             T(2.0 / 3.0) * kmp * rho * (d_ux_x - d_uy_y) + T(2.0 / 3.0) * (d_mux_x - d_muy_y);
        Cc = -third * kappa * (d_ruy_x + d_rux_y) + third * kmp * rho * (d_uy_x + d_ux_y) +
             third * (d_muy_x + d_mux_y);
      } else {
        Ca = -kappa * (d_rux_x + d_ruy_y) + T(2) * kmp * rho * (d_ux_x + d_uy_y) +
             (T(3) - T(2) * X) * (d_mux_x + d_muy_y);
        Cb = -kappa * (d_rux_x - d_ruy_y) + T(2.0 / 3.0) * kmp * rho * (d_ux_x - d_uy_y) +
             (d_mux_x - d_muy_y);
        Cc = third * kmp * rho * (d_uy_x + d_ux_y);
      }
      if (FEAT & FEAT_DYNPHI) Ca -= T(2) * X * rho * rC.dphi;

      // equilibria (Eq. 18) minus those of the rest state
      const T m0 = phi * rho0 + rC.dm0;  // phi rho
      const T drho = rC.drho;
      const T uu = ux * ux + uy * uy;
      const T eq_e = (T(2) * kappa - T(4) * phi) * drho + T(3) * m0 * uu;
      const T eq_ep = (T(4) * phi - T(3) * kappa) * drho - T(3) * m0 * uu;
      const T qfac = eq2 ? -m0 : (kappa - T(2) * phi) * rho;  // phi rho (X - 2), or -phi rho (B2)
      const T eq_qx = qfac * ux, eq_qy = qfac * uy;
      const T eq_pxx = m0 * (ux * ux - uy * uy);
      const T eq_pxy = m0 * (ux * uy);

      // force moments (Eq. 19)
      const T uF = ux * Fx + uy * Fy;
      const T S1 = T(6) * uF;
      const T S7 = T(2) * (ux * Fx - uy * Fy);
      const T S8 = ux * Fy + uy * Fx;

      // relaxation (Eq. 16); conserved moments: m0+ = m0, j+ = j + F
      const T he = T(1) - T(0.5) * ph.s_e, hep = T(1) - T(0.5) * ph.s_eps;
      const T hq = T(1) - T(0.5) * ph.s_q, hn = T(1) - T(0.5) * ph.s_nu;
      const T pe = rC.me - ph.s_e * (rC.me - eq_e) + he * (S1 + Ca);
      const T pep = rC.mep - ph.s_eps * (rC.mep - eq_ep) - hep * S1;
      const T pqx = rC.mqx - ph.s_q * (rC.mqx - eq_qx) - hq * Fx;
      const T pqy = rC.mqy - ph.s_q * (rC.mqy - eq_qy) - hq * Fy;
      const T ppxx = rC.mpxx - ph.s_nu * (rC.mpxx - eq_pxx) + hn * (S7 + Cb);
      const T ppxy = rC.mpxy - ph.s_nu * (rC.mpxy - eq_pxy) + hn * (S8 + Cc);
      const T pm0 = rC.dm0;
      const T pjx = rC.jx + Fx;
      const T pjy = rC.jy + Fy;

      // back-transform f+ = M^-1 m+ (Eq. A1)
      const T a = (T(4) * pm0 - pe - T(2) * pep) * T(1.0 / 36.0);
      const T b = (T(4) * pm0 + T(2) * pe + pep) * T(1.0 / 36.0);
      const T X1 = (pjx - pqx) * T(1.0 / 6.0), Y1 = (pjy - pqy) * T(1.0 / 6.0);
      const T X2 = (T(2) * pjx + pqx) * T(1.0 / 12.0), Y2 = (T(2) * pjy + pqy) * T(1.0 / 12.0);
      const T Pd = ppxx * T(0.25), Qd = ppxy * T(0.25);
      T o9[9];
      o9[0] = (pm0 - pe + pep) * T(1.0 / 9.0);
      o9[1] = a + X1 + Pd;
      o9[2] = a + Y1 - Pd;
      o9[3] = a - X1 + Pd;
      o9[4] = a - Y1 - Pd;
      o9[5] = b + X2 + Y2 + Qd;
      o9[6] = b - X2 + Y2 - Qd;
      o9[7] = b - X2 - Y2 + Qd;
      o9[8] = b + X2 - Y2 - Qd;
      if constexpr ((FEAT & FEAT_MASK) != 0) {  // solid node: keep the rest state
        if (solid_bit(rC.nb, 0)) {
#pragma unroll
          for (int i = 0; i < 9; ++i) o9[i] = T(0);
        }
      }
      // Store deviations o (rest state of void fraction ph_n) on row r.
      // Shifted storage holds deviations from the rest state of the void
      // fraction of the time the next pull runs at: rest_0 changes by
      // rho0 d_t phi when phi moves (dph_n).
      auto store_row = [&](T (&o)[9], T ph_n, T dph_n, int r) {
        if (SHIFT && (FEAT & FEAT_DYNPHI)) o[0] -= rho0 * dph_n;
        if (SHIFT) {
#pragma unroll
          for (int i = 0; i < 9; ++i)
            bstore(static_cast<S>(sizeof(S) == 2 ? o[i] * ph.scale : o[i]), dstr, xcb, poff(i, r));
        } else {
          bstore(static_cast<S>(o[0] + (ph_n * rho0 - ph.rest0_k)), dstr, xcb, poff(0, r));
#pragma unroll
          for (int i = 1; i < 5; ++i) bstore(static_cast<S>(o[i] + ph.rest_axis), dstr, xcb, poff(i, r));
#pragma unroll
          for (int i = 5; i < 9; ++i) bstore(static_cast<S>(o[i] + ph.rest_diag), dstr, xcb, poff(i, r));
        }
      };

      if constexpr (NEE) {
        // Velocity rows (Sec. 3.1: non-equilibrium extrapolation for the
        // moving wall of Couette flow).  The fluid row next to a velocity row
        // also sets that row's post-collision state,
        //   f+(x_b) = f^eq(phi_b, rho_f, u_w) + f+(x_f) - f^eq(phi_f, rho_f, u_f),
        // here on deviations; the velocity row itself stores nothing.
        auto vel_row = [&](int rb, T uw) {
          const unsigned ro = unsigned(rb) * unsigned(pitch) * TB;
          const T phb = bload<T>(phir, xcT, ro);
          const T dphb = (FEAT & FEAT_DYNPHI) ? bload<T>(phinr, xcT, ro) - phb : T(0);
          T ob[9];
          ob[0] = o9[0] + (eq_dev<0>(phb, rho, drho, uw, T(0), kappa, eq2) - eq_dev<0>(phi, rho, drho, ux, uy, kappa, eq2));
          ob[1] = o9[1] + (eq_dev<1>(phb, rho, drho, uw, T(0), kappa, eq2) - eq_dev<1>(phi, rho, drho, ux, uy, kappa, eq2));
          ob[2] = o9[2] + (eq_dev<2>(phb, rho, drho, uw, T(0), kappa, eq2) - eq_dev<2>(phi, rho, drho, ux, uy, kappa, eq2));
          ob[3] = o9[3] + (eq_dev<3>(phb, rho, drho, uw, T(0), kappa, eq2) - eq_dev<3>(phi, rho, drho, ux, uy, kappa, eq2));
          ob[4] = o9[4] + (eq_dev<4>(phb, rho, drho, uw, T(0), kappa, eq2) - eq_dev<4>(phi, rho, drho, ux, uy, kappa, eq2));
          ob[5] = o9[5] + (eq_dev<5>(phb, rho, drho, uw, T(0), kappa, eq2) - eq_dev<5>(phi, rho, drho, ux, uy, kappa, eq2));
          ob[6] = o9[6] + (eq_dev<6>(phb, rho, drho, uw, T(0), kappa, eq2) - eq_dev<6>(phi, rho, drho, ux, uy, kappa, eq2));
          ob[7] = o9[7] + (eq_dev<7>(phb, rho, drho, uw, T(0), kappa, eq2) - eq_dev<7>(phi, rho, drho, ux, uy, kappa, eq2));
          ob[8] = o9[8] + (eq_dev<8>(phb, rho, drho, uw, T(0), kappa, eq2) - eq_dev<8>(phi, rho, drho, ux, uy, kappa, eq2));
          store_row(ob, phb, dphb, rb);
        };
        if (ph.nee_lo && yo == 1) vel_row(0, ph.un_lo);
        if (ph.nee_hi && yo == ny - 2) vel_row(ny - 1, ph.un_hi);
        if ((ph.nee_lo && yo == 0) || (ph.nee_hi && yo == ny - 1)) return;
      }
      store_row(o9, phi, rC.dphi, yo);
    }
  };

  // Software pipeline: the loads of row yn+PD are in flight while row yn is
  // processed.  Unrolled by six so that the load buffers (period PD+1) and
  // the three row states (period 3) are renamed instead of copied.
  RowState<T> R0{}, R1{}, R2{};
  T b0[2] = {0, 0}, b1[2] = {0, 0};
  if constexpr (PD == 1) {
    RowIn<S, T> ia{}, ib{};
    load_row(y0 - 2, ia);
    for (int k = 0; k < nit; k += 6) {
      load_row(y0 - 1 + k, ib);
      body(k + 0, ia, R0, R2, R1, b0, b1);
      if (k + 1 >= nit) break;
      load_row(y0 + k, ia);
      body(k + 1, ib, R1, R0, R2, b1, b0);
      if (k + 2 >= nit) break;
      load_row(y0 + 1 + k, ib);
      body(k + 2, ia, R2, R1, R0, b0, b1);
      if (k + 3 >= nit) break;
      load_row(y0 + 2 + k, ia);
      body(k + 3, ib, R0, R2, R1, b1, b0);
      if (k + 4 >= nit) break;
      load_row(y0 + 3 + k, ib);
      body(k + 4, ia, R1, R0, R2, b0, b1);
      if (k + 5 >= nit) break;
      load_row(y0 + 4 + k, ia);
      body(k + 5, ib, R2, R1, R0, b1, b0);
    }
  } else {
    static_assert(PD == 2, "prefetch distance 1 or 2");
    RowIn<S, T> ia{}, ib{}, ic{};
    load_row(y0 - 2, ia);
    load_row(y0 - 1, ib);
    for (int k = 0; k < nit; k += 6) {
      load_row(y0 + k, ic);
      body(k + 0, ia, R0, R2, R1, b0, b1);
      if (k + 1 >= nit) break;
      load_row(y0 + 1 + k, ia);
      body(k + 1, ib, R1, R0, R2, b1, b0);
      if (k + 2 >= nit) break;
      load_row(y0 + 2 + k, ib);
      body(k + 2, ic, R2, R1, R0, b0, b1);
      if (k + 3 >= nit) break;
      load_row(y0 + 3 + k, ic);
      body(k + 3, ia, R0, R2, R1, b1, b0);
      if (k + 4 >= nit) break;
      load_row(y0 + 4 + k, ia);
      body(k + 4, ib, R1, R0, R2, b0, b1);
      if (k + 5 >= nit) break;
      load_row(y0 + 5 + k, ib);
      body(k + 5, ic, R2, R1, R0, b1, b0);
    }
  }
}

// One lattice per launch: workgroup b takes tile xcd_tile(b) (strip
// tile % strips, row block tile / strips).  WPE: minimum waves per SIMD the register allocation allows
// (three for the FP32 kernels with solid nodes and a moving phi or scheme
// variant, whose extra state would spill heavily at four; with solid nodes
// alone or with the force field and drag a few registers spill at four,
// which measures faster than three).
template <typename S, typename T, bool SHIFT, bool WALLS, int FEAT, int NT, int PD = 1,
          int WPE = (sizeof(T) == 4 ? (((FEAT & FEAT_MASK) && (FEAT & (FEAT_DYNPHI | FEAT_SCHEME))) ? 3 : 4) : 2)>
__global__ void __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(WPE)))
vanse_step_kernel(StepGeom g, StepPhys<T> ph) {
  __shared__ StepLds<T, NT> lds;
  const int tile = xcd_tile(int(blockIdx.x), int(gridDim.x));
  step_tile<S, T, SHIFT, WALLS, FEAT, NT, PD>(g, ph, tile % g.strips, tile / g.strips, lds);
}

// Many independent lattices per launch.  Entry xcd_tile(b) of the tile map
// gives workgroup b its lattice and the tile's index within that lattice
// (strip local % strips, row block local / strips); the host orders the map
// so that workgroups, in launch order, take the tiles with the most rows
// first.  The two population buffers of a lattice alternate with parity
// (cur0_k + launch) & 1.
template <typename T>
struct BatchEntry {
  StepGeom g;          // src/dst hold buffer 0 and buffer 1
  StepPhys<T> ph;
  int first_tile;
  int cur0;            // buffer holding the state before launch 0
};

template <typename S, typename T, bool SHIFT, bool WALLS, int FEAT, int NT,
          int WPE = (sizeof(T) == 4 ? (((FEAT & FEAT_MASK) && (FEAT & (FEAT_DYNPHI | FEAT_SCHEME))) ? 3 : 4) : 2)>
__global__ void __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(WPE)))
vanse_batch_step_kernel(const BatchEntry<T>* __restrict__ entries,
                        const int2* __restrict__ tile_map, int launch) {
  __shared__ StepLds<T, NT> lds;
  const int2 tm = tile_map[xcd_tile(int(blockIdx.x), int(gridDim.x))];
  const int k = tm.x;
  const BatchEntry<T>& e = entries[k];
  StepGeom g = e.g;
  const int par = (e.cur0 + launch) & 1;
  void* const b0 = const_cast<void*>(e.g.src);
  void* const b1 = e.g.dst;
  g.src = par ? b1 : b0;
  g.dst = par ? b0 : b1;
  const int local = tm.y;
  // a private copy, as the one-lattice kernel's argument (read through the
  // table the parameters could alias the stores as far as the compiler knows)
  const StepPhys<T> ph = e.ph;
  step_tile<S, T, SHIFT, WALLS, FEAT, NT, 1>(g, ph, local % g.strips, local / g.strips, lds);
}

}  // namespace vanse_dev
