// aux_kernels.hpp -- set-up and read-out kernels around the fused step:
// field uploads, initial populations, population I/O, macroscopic fields and
// FP64 observables.  None of these is on the per-step path.
//
// Storage convention (see step_kernel.hpp): buffer slot s_i(y) holds the
// post-collision population that the next pull delivers to node y + e_i as
// f_i, or -- when y + e_i lies beyond a wall -- back to node y as f_opp(i).
// Values are f (plain storage) or deviations g = f - f^rest (shifted storage,
// times a power-of-two scale).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "step_kernel.hpp"

namespace vanse_dev {

__constant__ int kEX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__constant__ int kEY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__constant__ int kOPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

struct Geo {
  int nx, ny, pitch, walls;
  int xwalls;  // half-way walls at x = -1/2 and x = nx - 1/2 as well
  long long plane;
  int nee_lo, nee_hi;  // velocity boundary rows (first / last row), see StepPhys
  double un_lo, un_hi;
};

// Kind of row y: 1 (2) when it is the lower (upper) velocity boundary row.
__device__ __forceinline__ int vel_row_kind(const Geo& G, int y) {
  if (!G.walls) return 0;
  if (G.nee_lo && y == 0) return 1;
  if (G.nee_hi && y == G.ny - 1) return 2;
  return 0;
}

constexpr int NOBS = 5;  // observables per reduction record

// Rest-state population f^rest_i = f^eq_i(rho0, 0) of Eq. (14) at a node
// of void fraction phi.
template <typename T>
__device__ __forceinline__ T rest_pop(int i, T phi, const StepPhys<T>& ph) {
  if (i == 0) return phi * ph.rho0 - ph.rest0_k;
  return (i < 5) ? ph.rest_axis : ph.rest_diag;
}

// Adjusted equilibrium of Eq. (14), written with cs^2 = 1/3 and X = kappa/phi:
// the third-order factor is (3 - X)/2 on the axes and X on the diagonals; 1
// for the second-order equilibrium of Eq. (B1) (eq2).
__device__ inline double feq_pop(int i, double phi, double rho, double ux, double uy,
                                 double kappa, int eq2) {
  const double uu = ux * ux + uy * uy;
  if (i == 0) return phi * rho - 5.0 / 9.0 * kappa * rho - 2.0 / 3.0 * phi * rho * uu;
  const double X = kappa / phi;
  const double eu = kEX[i] * ux + kEY[i] * uy;
  const bool axis = i < 5;
  const double w = axis ? 1.0 / 9.0 : 1.0 / 36.0;
  const double h3 = eq2 ? 1.0 : (axis ? 0.5 * (3.0 - X) : X);
  return w * (kappa * rho + phi * rho * (3.0 * eu * h3 + 4.5 * eu * eu - 1.5 * uu));
}

// Moving-wall correction of a population f+_i that crossed the wall at
// y = -1/2 (lo) or y = ny - 1/2 (hi): it returns as f_opp(i) = f+_i - delta,
// delta = f^eq_i - f^eq_opp(i) at (phi, rho0, u_w).
template <typename T>
__device__ inline double wall_delta(int i, T phi, bool lo, const StepPhys<T>& ph) {
  const double uw = double(lo ? ph.uw_lo : ph.uw_hi);
  if (uw == 0.0) return 0.0;
  return feq_pop(i, double(phi), double(ph.rho0), uw, 0.0, double(ph.kappa), ph.eq2) -
         feq_pop(kOPP[i], double(phi), double(ph.rho0), uw, 0.0, double(ph.kappa), ph.eq2);
}

template <typename S, typename T, bool SHIFT>
__device__ __forceinline__ S encode(double f, T phi, int i, const StepPhys<T>& ph) {
  if (SHIFT) return static_cast<S>((static_cast<T>(f - double(rest_pop(i, phi, ph)))) * ph.scale);
  return static_cast<S>(f);
}

template <typename S, typename T, bool SHIFT>
__device__ __forceinline__ double decode(S s, T phi, int i, const StepPhys<T>& ph) {
  if (SHIFT) return double(static_cast<T>(s) * ph.inv_scale) + double(rest_pop(i, phi, ph));
  return double(static_cast<T>(s));
}

// Solid flags of a node (0 without a mask); bit layout as FEAT_MASK.
__device__ __forceinline__ unsigned nbr_at(const Geo& G, const uint16_t* __restrict__ nbr, int x,
                                           int y) {
  return nbr ? unsigned(nbr[(long long)y * G.pitch + x]) : 0u;
}

// Receiving node of stored slot (x, y, i): (x + e_i, y + e_i) or, across a
// wall or onto a solid node (flag bit i), (x, y) with direction opp(i).
// Returns false for the bounce-back case.
__device__ __forceinline__ bool receiver(const Geo& G, int x, int y, int i, unsigned nb, int* xr,
                                         int* yr) {
  int xn = x + kEX[i];
  int yn = y + kEY[i];
  if (G.xwalls && (xn < 0 || xn >= G.nx)) { *xr = x; *yr = y; return false; }
  xn = xn < 0 ? xn + G.nx : (xn >= G.nx ? xn - G.nx : xn);
  if (G.walls) {
    if (yn < 0 || yn >= G.ny) { *xr = x; *yr = y; return false; }
  } else {
    yn = yn < 0 ? yn + G.ny : (yn >= G.ny ? yn - G.ny : yn);
  }
  if (i > 0 && solid_bit(nb, i)) { *xr = x; *yr = y; return false; }
  *xr = xn; *yr = yn;
  return true;
}

// Solid flags (FEAT_MASK layout) from a dense uint8 mask, nonzero = solid:
// bit 0 the node, bit i the node standing in for x + e_i, which across a wall
// is its mirror image in the first or last row (or column).  A solid node
// keeps bit 0 alone: nothing it computes is used, and without neighbour bits
// the step's bounce-back and stand-in paths pass over solid regions.  Counts
// solid nodes.
__global__ void build_nbr(Geo G, const uint8_t* __restrict__ mask, uint16_t* __restrict__ nbr,
                          unsigned long long* __restrict__ nsolid) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= G.nx || y >= G.ny) return;
  unsigned b = mask[(long long)y * G.nx + x] ? 1u : 0u;
  for (int i = 1; i < 9; ++i) {
    int xn = x + kEX[i], yn = y + kEY[i];
    if (G.xwalls) xn = xn < 0 ? -1 - xn : (xn >= G.nx ? 2 * G.nx - 1 - xn : xn);
    else xn = xn < 0 ? xn + G.nx : (xn >= G.nx ? xn - G.nx : xn);
    if (G.walls) yn = yn < 0 ? -1 - yn : (yn >= G.ny ? 2 * G.ny - 1 - yn : yn);
    else yn = yn < 0 ? yn + G.ny : (yn >= G.ny ? yn - G.ny : yn);
    if (mask[(long long)yn * G.nx + xn]) b |= 1u << i;
  }
  if (b & 1u) b = 1u;
  nbr[(long long)y * G.pitch + x] = (uint16_t)b;
  if (b & 1u) atomicAdd(nsolid, 1ull);
}

// phi = 1 on solid nodes (a finite placeholder; never enters a fluid node).
template <typename T>
__global__ void phi_on_solids(Geo G, T* __restrict__ phi, const uint16_t* __restrict__ nbr) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= G.nx || y >= G.ny) return;
  if (nbr[(long long)y * G.pitch + x] & 1u) phi[(long long)y * G.pitch + x] = T(1);
}

// Convert a dense float64 field to a pitched plane of T.
template <typename T>
__global__ void convert_field(const double* __restrict__ in, T* __restrict__ out, int nx, int ny,
                              int pitch) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x < nx && y < ny) out[y * pitch + x] = static_cast<T>(in[y * nx + x]);
}

// Count entries of a dense field outside (0, 1] (or non-finite), solid
// nodes (flag bit 0 of nbr, when given) excepted.
__global__ void count_bad_phi(const double* __restrict__ in, int nx, long long n,
                              const uint16_t* __restrict__ nbr, int pitch,
                              unsigned long long* __restrict__ bad) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  unsigned long long cnt = 0;
  for (; i < n; i += stride) {
    if (nbr && (nbr[(i / nx) * pitch + i % nx] & 1u)) continue;
    const double v = in[i];
    if (!(v > 0.0 && v <= 1.0)) ++cnt;
  }
  if (cnt) atomicAdd(bad, cnt);
}

// Fill the stored slots so that the next pull yields f(0): either the
// equilibrium of Eq. (14) at (rho0, u0), or given dense populations.
template <typename S, typename T, bool SHIFT>
__global__ void fill_state(Geo G, S* __restrict__ buf, const T* __restrict__ phi, StepPhys<T> ph,
                           const double* __restrict__ fin, double rho_init, double ux0, double uy0,
                           double kappa, const uint16_t* __restrict__ nbr) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= G.nx || y >= G.ny) return;
  const long long N = (long long)G.nx * G.ny;
  const unsigned nb = nbr_at(G, nbr, x, y);
  if (nb & 1u) {  // solid node: the rest state (never pulled by a fluid node)
    const T ph_x = phi[y * G.pitch + x];
    for (int i = 0; i < 9; ++i)
      buf[i * G.plane + (long long)y * G.pitch + x] =
          encode<S, T, SHIFT>(double(rest_pop(i, ph_x, ph)), ph_x, i, ph);
    return;
  }
  for (int i = 0; i < 9; ++i) {
    int xr, yr;
    const bool through = receiver(G, x, y, i, nb, &xr, &yr);
    const int j = through ? i : kOPP[i];  // population index at the receiver
    const T phr = phi[yr * G.pitch + xr];
    double f;
    if (fin) {
      f = fin[j * N + (long long)yr * G.nx + xr];
    } else {
      f = feq_pop(j, double(phr), rho_init, ux0, uy0, kappa, ph.eq2);
    }
    const int yn = y + kEY[i];
    if (!through && G.walls && (yn < 0 || yn >= G.ny))  // the pull subtracts it again
      f += wall_delta(i, phr, yn < 0, ph);
    buf[i * G.plane + (long long)y * G.pitch + x] = encode<S, T, SHIFT>(f, phr, j, ph);
  }
}

// Pull the populations of the current time: f_i(x) = slot_i(x - e_i), or
// slot_opp(i)(x) when x - e_i is beyond a wall or solid (flag bit opp(i)).
template <typename S, typename T, bool SHIFT>
__device__ __forceinline__ double pull_one(const Geo& G, const S* __restrict__ buf, T phi_x,
                                           const StepPhys<T>& ph, int x, int y, int i,
                                           unsigned nb) {
  int xs = x - kEX[i];
  int ys = y - kEY[i];
  int slot = i;
  const bool xout = xs < 0 || xs >= G.nx;
  xs = xs < 0 ? xs + G.nx : (xs >= G.nx ? xs - G.nx : xs);
  double corr = 0.0;
  if (G.walls && (ys < 0 || ys >= G.ny)) {
    corr = wall_delta(kOPP[i], phi_x, ys < 0, ph);
    xs = x; ys = y; slot = kOPP[i];
  } else if (i > 0 && (solid_bit(nb, kOPP[i]) || (G.xwalls && xout))) {
    xs = x; ys = y; slot = kOPP[i];
  } else {
    ys = ys < 0 ? ys + G.ny : (ys >= G.ny ? ys - G.ny : ys);
  }
  const S s = buf[slot * G.plane + (long long)ys * G.pitch + xs];
  // rest_i depends on phi only for i = 0
  return decode<S, T, SHIFT>(s, phi_x, i, ph) - corr;
}

// Populations f_i(x, t); zero on solid nodes.
template <typename S, typename T, bool SHIFT>
__global__ void read_pops(Geo G, const S* __restrict__ buf, const T* __restrict__ phi,
                          StepPhys<T> ph, double* __restrict__ out,
                          const uint16_t* __restrict__ nbr) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= G.nx || y >= G.ny) return;
  const long long N = (long long)G.nx * G.ny;
  const T ph_x = phi[y * G.pitch + x];
  const unsigned nb = nbr_at(G, nbr, x, y);
  for (int i = 0; i < 9; ++i)
    out[i * N + (long long)y * G.nx + x] =
        (nb & 1u) ? 0.0 : pull_one<S, T, SHIFT>(G, buf, ph_x, ph, x, y, i, nb);
}

// delta rho = sum_i (f_i - rest_i) / phi of node (x, y), in T; a velocity
// row takes the density of the fluid row next to it; 0 on a solid node.
template <typename S, typename T, bool SHIFT>
__device__ __forceinline__ T node_drho(const Geo& G, const S* __restrict__ buf,
                                       const T* __restrict__ phi, const StepPhys<T>& ph, int x,
                                       int y, const uint16_t* __restrict__ nbr) {
  const int kind = vel_row_kind(G, y);
  const int ys = kind == 1 ? 1 : (kind == 2 ? G.ny - 2 : y);
  const T ph_x = phi[ys * G.pitch + x];
  const unsigned nb = nbr_at(G, nbr, x, ys);
  T dm0 = 0;
  for (int i = 0; i < 9; ++i) {
    const double f = pull_one<S, T, SHIFT>(G, buf, ph_x, ph, x, ys, i, nb);
    dm0 += static_cast<T>(f - double(rest_pop(i, ph_x, ph)));
  }
  return (nb & 1u) ? T(0) : dm0 / ph_x;
}

// Pass 1 of the macroscopic read-out: delta rho (in T) to a scratch plane.
template <typename S, typename T, bool SHIFT>
__global__ void moments_rho(Geo G, const S* __restrict__ buf, const T* __restrict__ phi,
                            StepPhys<T> ph, T* __restrict__ drho_out,
                            const uint16_t* __restrict__ nbr) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= G.nx || y >= G.ny) return;
  drho_out[y * G.pitch + x] = node_drho<S, T, SHIFT>(G, buf, phi, ph, x, y, nbr);
}

// Pass 2: grad rho (Eq. 10 with mirror images at walls and centre values for
// solid neighbours), F, u, p; optional FP64 block partials of the
// observables.  Solid nodes report zeros and are left out of the partials.
// delta rho of the node and its neighbours comes from the plane of pass 1,
// or (drho = null) is formed again from their populations, so that the
// observables need no scratch plane.
template <typename S, typename T, bool SHIFT, int FEAT>
__global__ void moments_out(Geo G, const S* __restrict__ buf, const T* __restrict__ phi,
                            StepPhys<T> ph, const T* __restrict__ drho, const T* __restrict__ fxf,
                            const T* __restrict__ fyf, const T* __restrict__ beta,
                            double* __restrict__ rho_o,
                            double* __restrict__ ux_o, double* __restrict__ uy_o,
                            double* __restrict__ p_o, double* __restrict__ partials,
                            T* __restrict__ uprev, int uprev_valid,
                            const uint16_t* __restrict__ nbr) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  double mass = 0.0, u2 = 0.0, umax = 0.0, bad = 0.0, du2 = 0.0;
  const unsigned nb = (x < G.nx && y < G.ny) ? nbr_at(G, nbr, x, y) : 0u;
  const int vkind = (x < G.nx && y < G.ny) ? vel_row_kind(G, y) : 0;
  if (x < G.nx && y < G.ny && (nb & 1u)) {
    const long long o = (long long)y * G.nx + x;
    if (rho_o) rho_o[o] = 0.0;
    if (ux_o) ux_o[o] = 0.0;
    if (uy_o) uy_o[o] = 0.0;
    if (p_o) p_o[o] = 0.0;
  } else if (vkind) {
    // velocity row: the wall velocity and the fluid neighbour's density; not
    // a fluid node, so left out of the observables
    const long long o = (long long)y * G.nx + x;
    const double rho = double(ph.rho0 + (drho ? drho[y * G.pitch + x]
                                               : node_drho<S, T, SHIFT>(G, buf, phi, ph, x, y, nbr)));
    if (rho_o) rho_o[o] = rho;
    if (ux_o) ux_o[o] = vkind == 1 ? G.un_lo : G.un_hi;
    if (uy_o) uy_o[o] = 0.0;
    if (p_o) p_o[o] = rho / 3.0;
  } else if (x < G.nx && y < G.ny) {
    const T ph_x = phi[y * G.pitch + x];
    double m0 = 0.0, jx = 0.0, jy = 0.0;
    T dm0 = 0;
    T f[9];
    for (int i = 0; i < 9; ++i) {
      const double fi = pull_one<S, T, SHIFT>(G, buf, ph_x, ph, x, y, i, nb);
      f[i] = static_cast<T>(fi - double(rest_pop(i, ph_x, ph)));
      m0 += fi;
    }
    for (int i = 0; i < 9; ++i) dm0 += f[i];
    T tjx = (f[1] - f[3]) + ((f[5] - f[6]) + (f[8] - f[7]));
    T tjy = (f[2] - f[4]) + ((f[5] + f[6]) - (f[7] + f[8]));
    jx = tjx; jy = tjy;
    // neighbours of delta-rho (direction i of Eq. 5); mirror image across
    // walls, the centre value for a solid neighbour
    auto drho_at = [&](int xq, int yq) -> T {
      return drho ? drho[yq * G.pitch + xq] : node_drho<S, T, SHIFT>(G, buf, phi, ph, xq, yq, nbr);
    };
    const T rc = drho_at(x, y);
    auto R = [&](int i) -> T {
      if (solid_bit(nb, i)) return rc;
      int xn = x + kEX[i], yn = y + kEY[i];
      if (G.xwalls) xn = xn < 0 ? 0 : (xn >= G.nx ? G.nx - 1 : xn);
      else xn = xn < 0 ? xn + G.nx : (xn >= G.nx ? xn - G.nx : xn);
      if (G.walls) {
        yn = yn < 0 ? 0 : (yn >= G.ny ? G.ny - 1 : yn);
      } else {
        yn = yn < 0 ? yn + G.ny : (yn >= G.ny ? yn - G.ny : yn);
      }
      return drho_at(xn, yn);
    };
    const T grx = stencil_dx(R(1), R(3), R(5), R(8), R(6), R(7));
    const T gry = stencil_dy(R(2), R(4), R(5), R(6), R(8), R(7));
    const T kp = (ph.kappa - (ph.model_b ? T(1) : ph_x)) * T(1.0 / 3.0);  // Eq. (13) / model B
    const T sg = ph.scale_by_phi ? ph_x : T(1);
    T Fx = kp * grx + sg * ph.gx;
    T Fy = kp * gry + sg * ph.gy;
    if ((FEAT & FEAT_FORCE) && fxf) {
      Fx += fxf[y * G.pitch + x];
      Fy += fyf[y * G.pitch + x];
    }
    const T tm0 = ph_x * ph.rho0 + dm0;
    T ux, uy;
    if ((FEAT & FEAT_DRAG) && beta) {  // u of Eq. (7) with the drag solved in closed form
      const T d = ph_x * beta[y * G.pitch + x];
      ux = (tjx + T(0.5) * (Fx + d * ph.usx)) / (tm0 + T(0.5) * d);
      uy = (tjy + T(0.5) * (Fy + d * ph.usy)) / (tm0 + T(0.5) * d);
    } else {
      ux = (tjx + T(0.5) * Fx) / tm0;
      uy = (tjy + T(0.5) * Fy) / tm0;
    }
    const T rho = ph.rho0 + dm0 / ph_x;
    const long long o = (long long)y * G.nx + x;
    if (rho_o) rho_o[o] = double(rho);
    if (ux_o) ux_o[o] = double(ux);
    if (uy_o) uy_o[o] = double(uy);
    if (p_o) p_o[o] = double(rho) / 3.0;
    if (uprev) {  // |u(t) - u(t')|^2 against the velocity kept at the last call
      T* px = uprev + (long long)y * G.pitch + x;
      T* py = px + G.plane;
      if (uprev_valid) {
        const double dx = double(ux) - double(*px), dy = double(uy) - double(*py);
        du2 = dx * dx + dy * dy;
      }
      *px = ux;
      *py = uy;
    }
    mass = m0;
    u2 = double(ux) * double(ux) + double(uy) * double(uy);
    umax = sqrt(u2);
    const bool finite = isfinite(m0) && isfinite(double(ux)) && isfinite(double(uy)) &&
                        isfinite(jx) && isfinite(jy);
    bad = finite ? 0.0 : 1.0;
    if (!finite) { mass = 0.0; u2 = 0.0; umax = 0.0; du2 = 0.0; }
  }
  if (partials) {
    // block reduction in a fixed order: wavefront shuffles, then LDS
    __shared__ double red[NOBS][16];
    for (int off = 32; off > 0; off >>= 1) {
      mass += __shfl_down(mass, off, 64);
      u2 += __shfl_down(u2, off, 64);
      umax = fmax(umax, __shfl_down(umax, off, 64));
      bad += __shfl_down(bad, off, 64);
      du2 += __shfl_down(du2, off, 64);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
      red[0][wv] = mass; red[1][wv] = u2; red[2][wv] = umax; red[3][wv] = bad; red[4][wv] = du2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int nw = blockDim.x >> 6;
      double a[NOBS] = {0, 0, 0, 0, 0};
      for (int k = 0; k < nw; ++k) {
        a[0] += red[0][k]; a[1] += red[1][k]; a[2] = fmax(a[2], red[2][k]); a[3] += red[3][k];
        a[4] += red[4][k];
      }
      const long long blk = (long long)blockIdx.y * gridDim.x + blockIdx.x;
      for (int q = 0; q < NOBS; ++q) partials[blk * NOBS + q] = a[q];
    }
  }
}

// Fixed-order reduction of block partials, in two levels: reduce_partials
// folds contiguous chunks (one workgroup per chunk) and is applied again to
// the chunk results until one record is left.  Record fields: mass, sum |u|^2,
// max |u|, non-finite count, sum |u - u_prev|^2.
__global__ void reduce_partials(const double* __restrict__ partials, long long nblk,
                                long long chunk, double* __restrict__ out) {
  __shared__ double red[NOBS][256];
  const long long beg = (long long)blockIdx.x * chunk;
  const long long end = min(beg + chunk, nblk);
  double a[NOBS] = {0, 0, 0, 0, 0};
  for (long long k = beg + threadIdx.x; k < end; k += blockDim.x) {
    a[0] += partials[k * NOBS + 0];
    a[1] += partials[k * NOBS + 1];
    a[2] = fmax(a[2], partials[k * NOBS + 2]);
    a[3] += partials[k * NOBS + 3];
    a[4] += partials[k * NOBS + 4];
  }
  for (int q = 0; q < NOBS; ++q) red[q][threadIdx.x] = a[q];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
      red[2][threadIdx.x] = fmax(red[2][threadIdx.x], red[2][threadIdx.x + s]);
      red[3][threadIdx.x] += red[3][threadIdx.x + s];
      red[4][threadIdx.x] += red[4][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < NOBS; ++q) out[(long long)blockIdx.x * NOBS + q] = red[q][0];
}

// In-step divergence check: reset the flag (first time a non-finite node was
// seen, -1 for none) ...
__global__ void set_flag(long long* __restrict__ flag, long long v) {
  if (threadIdx.x == 0) *flag = v;
}

// ... and record time t in it when the reduced observables (record field 3,
// the non-finite count) show a non-finite node and no earlier check did.
__global__ void note_nonfinite(const double* __restrict__ rec, long long t,
                               long long* __restrict__ flag) {
  if (threadIdx.x == 0 && rec[3] > 0.0 && *flag < 0) *flag = t;
}

// Speed-of-light reference with the step's memory pattern: every node pulls
// its nine populations from the same shifted positions (with the same
// bounce-back at walls) and writes them back unchanged to the other buffer.
// No arithmetic: 9 reads + 9 writes per node, the step's HBM traffic minus
// the phi plane.
template <typename S>
__global__ void __launch_bounds__(256) stream_copy(Geo G, const S* __restrict__ src,
                                                   S* __restrict__ dst) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= G.nx || y >= G.ny) return;
  const long long P = G.plane;
  const int xm = x == 0 ? G.nx - 1 : x - 1, xp = x == G.nx - 1 ? 0 : x + 1;
  const int o = y * G.pitch;
  S f[9];
  f[0] = src[o + x];
  f[1] = src[P + o + xm];
  f[3] = src[3 * P + o + xp];
  if (G.walls && y == 0) {
    f[2] = src[4 * P + o + x]; f[5] = src[7 * P + o + x]; f[6] = src[8 * P + o + x];
  } else {
    const int os = (y == 0 ? G.ny - 1 : y - 1) * G.pitch;
    f[2] = src[2 * P + os + x]; f[5] = src[5 * P + os + xm]; f[6] = src[6 * P + os + xp];
  }
  if (G.walls && y == G.ny - 1) {
    f[4] = src[2 * P + o + x]; f[7] = src[5 * P + o + x]; f[8] = src[6 * P + o + x];
  } else {
    const int on = (y == G.ny - 1 ? 0 : y + 1) * G.pitch;
    f[4] = src[4 * P + on + x]; f[7] = src[7 * P + on + xp]; f[8] = src[8 * P + on + xm];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) dst[i * P + o + x] = f[i];
}

}  // namespace vanse_dev
