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
//
// Work layout: one workgroup owns a strip of `out_w` columns plus two halo
// columns on each side (one lane per column) and sweeps a block of rows
// bottom-up.  Per sweep iteration three stages run on three consecutive rows:
//   A  row yn   : pull the 9 populations, moments, delta-rho -> LDS ring(5)
//   B  row yn-1 : grad rho from the ring, F and u -> LDS ring(3)
//   C  row yn-2 : the eight derivatives from the rings, collision, store.
// Populations of rows yn-1, yn-2 stay in registers between stages, so each
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

template <typename T>
struct alignas(4 * sizeof(T)) U4 {
  T ux, uy, mux, muy;  // u and (phi rho) u at one node
};

template <typename T>
struct StepPhys {
  T kappa, rho0;
  T gx, gy;                 // uniform acceleration G
  T s_e, s_eps, s_q, s_nu;  // relaxation rates (non-conserved moments)
  T rest_axis, rest_diag;   // w_i kappa rho0 for |e|=1 and |e|=sqrt2
  T rest0_k;                // 5 kappa rho0 / 9 : rest_0 = phi rho0 - rest0_k
  T scale, inv_scale;       // storage scale of shifted half storage
  int scale_by_phi;
};

struct StepGeom {
  const void* src;
  void* dst;
  const void* phi;
  const void* fxf;
  const void* fyf;
  long long plane;  // elements per population plane (= pitch * ny)
  int nx, ny, pitch;
  int strips, out_w, rows;
};

__device__ __forceinline__ int wrap_index(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

__device__ __forceinline__ int slot5(int y) { return (y + 10) % 5; }
__device__ __forceinline__ int slot3(int y) { return (y + 9) % 3; }

template <typename S, typename T>
__device__ __forceinline__ T load_pop(const S* p) {
  return static_cast<T>(*p);
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

// S: storage type of populations (double, float, _Float16)
// T: arithmetic type (double, float)
// SHIFT: memory holds deviations g (scaled by ph.scale) instead of f
// WALLS: half-way bounce-back walls at y = -1/2 and y = ny - 1/2
// FFIELD: add the per-node force planes to F^B
// NT: threads per workgroup (= out_w + 4 active lanes at most)
template <typename S, typename T, bool SHIFT, bool WALLS, bool FFIELD, int NT>
__global__ void __launch_bounds__(NT) vanse_step_kernel(StepGeom g, StepPhys<T> ph) {
  __shared__ T s_rho[5][NT];     // delta-rho of the last five pulled rows
  __shared__ U4<T> s_u[3][NT];   // u, (phi rho) u of the last three rows

  const int t = threadIdx.x;
  const int strip = blockIdx.x % g.strips;
  const int by = blockIdx.x / g.strips;
  const int nx = g.nx, ny = g.ny, pitch = g.pitch;
  const int x0 = strip * g.out_w;
  const int w = min(g.out_w, nx - x0);
  const bool live = t < w + 4;                 // pulls and delta-rho
  const bool ulane = t >= 1 && t < w + 3;      // velocity
  const bool olane = t >= 2 && t < w + 2;      // collision and store
  const int c = wrap_index(x0 - 2 + t, nx);
  const int cm = (c == 0) ? nx - 1 : c - 1;
  const int cp = (c == nx - 1) ? 0 : c + 1;
  const int tl = max(t - 1, 0), tr = min(t + 1, NT - 1);

  const S* __restrict__ src = static_cast<const S*>(g.src);
  S* __restrict__ dst = static_cast<S*>(g.dst);
  const T* __restrict__ phif = static_cast<const T*>(g.phi);
  const long long P = g.plane;

  const int y0 = by * g.rows;
  const int y1 = min(y0 + g.rows, ny);
  const int nit = (y1 - y0) + 4;

  const T kappa = ph.kappa, rho0 = ph.rho0;
  const T third = T(1.0 / 3.0);

  T gB[9], gC[9];                  // deviations of rows yn-1, yn-2
  T sB[5], sC[5];                  // dm0, jx, jy, phi, drho of rows yn-1, yn-2
  T bC[4] = {0, 0, 0, 0};          // ux, uy, Fx, Fy of row yn-2
#pragma unroll
  for (int i = 0; i < 9; ++i) { gB[i] = T(0); gC[i] = T(0); }
#pragma unroll
  for (int i = 0; i < 5; ++i) { sB[i] = T(0); sC[i] = T(0); }

  for (int k = 0; k < nit; ++k) {
    const int yn = y0 - 2 + k;
    T gA[9];
    T sA[5];
#pragma unroll
    for (int i = 0; i < 9; ++i) gA[i] = T(0);
#pragma unroll
    for (int i = 0; i < 5; ++i) sA[i] = T(0);

    // ---------------- stage A: pull row yn ----------------
    const bool rowA = WALLS ? (yn >= 0 && yn < ny) : true;
    if (rowA && live) {
      const int r = WALLS ? yn : wrap_index(yn, ny);
      const int rs = WALLS ? yn - 1 : wrap_index(yn - 1, ny);
      const int rn = WALLS ? yn + 1 : wrap_index(yn + 1, ny);
      const int o = r * pitch;
      const T phi = phif[o + c];
      T f[9];
      f[0] = load_pop<S, T>(src + 0 * P + o + c);
      f[1] = load_pop<S, T>(src + 1 * P + o + cm);
      f[3] = load_pop<S, T>(src + 3 * P + o + cp);
      if (WALLS && yn == 0) {  // sources below the lower wall: bounce back
        f[2] = load_pop<S, T>(src + 4 * P + o + c);
        f[5] = load_pop<S, T>(src + 7 * P + o + c);
        f[6] = load_pop<S, T>(src + 8 * P + o + c);
      } else {
        const int os = rs * pitch;
        f[2] = load_pop<S, T>(src + 2 * P + os + c);
        f[5] = load_pop<S, T>(src + 5 * P + os + cm);
        f[6] = load_pop<S, T>(src + 6 * P + os + cp);
      }
      if (WALLS && yn == ny - 1) {  // sources above the upper wall
        f[4] = load_pop<S, T>(src + 2 * P + o + c);
        f[7] = load_pop<S, T>(src + 5 * P + o + c);
        f[8] = load_pop<S, T>(src + 6 * P + o + c);
      } else {
        const int on = rn * pitch;
        f[4] = load_pop<S, T>(src + 4 * P + on + c);
        f[7] = load_pop<S, T>(src + 7 * P + on + cp);
        f[8] = load_pop<S, T>(src + 8 * P + on + cm);
      }
      if (SHIFT) {
#pragma unroll
        for (int i = 0; i < 9; ++i) gA[i] = f[i] * ph.inv_scale;
      } else {
        gA[0] = f[0] - (phi * rho0 - ph.rest0_k);
#pragma unroll
        for (int i = 1; i < 5; ++i) gA[i] = f[i] - ph.rest_axis;
#pragma unroll
        for (int i = 5; i < 9; ++i) gA[i] = f[i] - ph.rest_diag;
      }
      const T dm0 = gA[0] + ((gA[1] + gA[2]) + (gA[3] + gA[4])) +
                    ((gA[5] + gA[6]) + (gA[7] + gA[8]));
      const T jx = (gA[1] - gA[3]) + ((gA[5] - gA[6]) + (gA[8] - gA[7]));
      const T jy = (gA[2] - gA[4]) + ((gA[5] + gA[6]) - (gA[7] + gA[8]));
      const T drho = dm0 / phi;
      sA[0] = dm0; sA[1] = jx; sA[2] = jy; sA[3] = phi; sA[4] = drho;
      s_rho[slot5(yn)][t] = drho;
    }
    __syncthreads();

    // ---------------- stage B: velocity of row yn-1 ----------------
    const int yb = yn - 1;
    T bN[4] = {0, 0, 0, 0};
    const bool rowB = (yb >= y0 - 1) && (WALLS ? (yb >= 0 && yb < ny) : true);
    if (rowB && ulane) {
      const int sc = slot5(yb);
      const int ss = (WALLS && yb == 0) ? sc : slot5(yb - 1);       // mirror image
      const int sn = (WALLS && yb == ny - 1) ? sc : slot5(yb + 1);
      const T rE = s_rho[sc][tr], rW = s_rho[sc][tl];
      const T rN = s_rho[sn][t], rS = s_rho[ss][t];
      const T rNE = s_rho[sn][tr], rNW = s_rho[sn][tl];
      const T rSE = s_rho[ss][tr], rSW = s_rho[ss][tl];
      const T grx = stencil_dx(rE, rW, rNE, rSE, rNW, rSW);
      const T gry = stencil_dy(rN, rS, rNE, rNW, rSE, rSW);
      const T phi = sB[3];
      const T kp = (kappa - phi) * third;
      const T sg = ph.scale_by_phi ? phi : T(1);
      T Fx = kp * grx + sg * ph.gx;
      T Fy = kp * gry + sg * ph.gy;
      if (FFIELD) {
        const int r = WALLS ? yb : wrap_index(yb, ny);
        Fx += static_cast<const T*>(g.fxf)[r * pitch + c];
        Fy += static_cast<const T*>(g.fyf)[r * pitch + c];
      }
      const T m0 = phi * rho0 + sB[0];
      const T inv_m0 = T(1) / m0;
      const T ux = (sB[1] + T(0.5) * Fx) * inv_m0;
      const T uy = (sB[2] + T(0.5) * Fy) * inv_m0;
      U4<T> uu;
      uu.ux = ux; uu.uy = uy; uu.mux = m0 * ux; uu.muy = m0 * uy;
      s_u[slot3(yb)][t] = uu;
      bN[0] = ux; bN[1] = uy; bN[2] = Fx; bN[3] = Fy;
    }
    __syncthreads();

    // ---------------- stage C: collide row yn-2 ----------------
    const int yo = yn - 2;
    if (yo >= y0 && olane) {
      const bool lo_wall = WALLS && yo == 0;
      const bool hi_wall = WALLS && yo == ny - 1;
      const int uo = slot3(yo);
      const int us = lo_wall ? uo : slot3(yo - 1);
      const int un = hi_wall ? uo : slot3(yo + 1);
      const int ro = slot5(yo);
      const int rs = lo_wall ? ro : slot5(yo - 1);
      const int rn = hi_wall ? ro : slot5(yo + 1);
      const T sgs = lo_wall ? T(-1) : T(1);  // velocity images change sign
      const T sgn = hi_wall ? T(-1) : T(1);

      const U4<T> qE = s_u[uo][tr], qW = s_u[uo][tl];
      U4<T> qN = s_u[un][t], qS = s_u[us][t];
      U4<T> qNE = s_u[un][tr], qNW = s_u[un][tl];
      U4<T> qSE = s_u[us][tr], qSW = s_u[us][tl];
      const T pE = rho0 + s_rho[ro][tr], pW = rho0 + s_rho[ro][tl];
      const T pN = rho0 + s_rho[rn][t], pS = rho0 + s_rho[rs][t];
      const T pNE = rho0 + s_rho[rn][tr], pNW = rho0 + s_rho[rn][tl];
      const T pSE = rho0 + s_rho[rs][tr], pSW = rho0 + s_rho[rs][tl];
      qN.ux *= sgn; qN.uy *= sgn; qN.mux *= sgn; qN.muy *= sgn;
      qNE.ux *= sgn; qNE.uy *= sgn; qNE.mux *= sgn; qNE.muy *= sgn;
      qNW.ux *= sgn; qNW.uy *= sgn; qNW.mux *= sgn; qNW.muy *= sgn;
      qS.ux *= sgs; qS.uy *= sgs; qS.mux *= sgs; qS.muy *= sgs;
      qSE.ux *= sgs; qSE.uy *= sgs; qSE.mux *= sgs; qSE.muy *= sgs;
      qSW.ux *= sgs; qSW.uy *= sgs; qSW.mux *= sgs; qSW.muy *= sgs;

      // the eight derivatives of Eq. (20), each by Eq. (10)
      const T d_rux_x = stencil_dx(pE * qE.ux, pW * qW.ux, pNE * qNE.ux, pSE * qSE.ux,
                                   pNW * qNW.ux, pSW * qSW.ux);
      const T d_ruy_y = stencil_dy(pN * qN.uy, pS * qS.uy, pNE * qNE.uy, pNW * qNW.uy,
                                   pSE * qSE.uy, pSW * qSW.uy);
      const T d_ux_x = stencil_dx(qE.ux, qW.ux, qNE.ux, qSE.ux, qNW.ux, qSW.ux);
      const T d_uy_y = stencil_dy(qN.uy, qS.uy, qNE.uy, qNW.uy, qSE.uy, qSW.uy);
      const T d_uy_x = stencil_dx(qE.uy, qW.uy, qNE.uy, qSE.uy, qNW.uy, qSW.uy);
      const T d_ux_y = stencil_dy(qN.ux, qS.ux, qNE.ux, qNW.ux, qSE.ux, qSW.ux);
      const T d_mux_x = stencil_dx(qE.mux, qW.mux, qNE.mux, qSE.mux, qNW.mux, qSW.mux);
      const T d_muy_y = stencil_dy(qN.muy, qS.muy, qNE.muy, qNW.muy, qSE.muy, qSW.muy);

      const T phi = sC[3];
      const T rho = rho0 + sC[4];
      const T X = kappa / phi;
      const T kmp = kappa - phi;
      const T ux = bC[0], uy = bC[1], Fx = bC[2], Fy = bC[3];

      // penalty source (Eq. 20); d_t phi = 0 for a static void fraction
      const T Ca = -kappa * (d_rux_x + d_ruy_y) + T(2) * kmp * rho * (d_ux_x + d_uy_y) +
                   (T(3) - T(2) * X) * (d_mux_x + d_muy_y);
      const T Cb = -kappa * (d_rux_x - d_ruy_y) + T(2.0 / 3.0) * kmp * rho * (d_ux_x - d_uy_y) +
                   (d_mux_x - d_muy_y);
      const T Cc = third * kmp * rho * (d_uy_x + d_ux_y);

      // non-conserved moments of the deviations (rows of M, Eq. A1)
      const T* q = gC;
      const T sa = (q[1] + q[2]) + (q[3] + q[4]);
      const T sd = (q[5] + q[6]) + (q[7] + q[8]);
      const T me = T(-4) * q[0] - sa + T(2) * sd;
      const T mep = T(4) * q[0] - T(2) * sa + sd;
      const T mqx = T(-2) * (q[1] - q[3]) + ((q[5] - q[6]) + (q[8] - q[7]));
      const T mqy = T(-2) * (q[2] - q[4]) + ((q[5] + q[6]) - (q[7] + q[8]));
      const T mpxx = (q[1] + q[3]) - (q[2] + q[4]);
      const T mpxy = (q[5] + q[7]) - (q[6] + q[8]);

      // equilibria (Eq. 18) minus those of the rest state
      const T m0 = phi * rho0 + sC[0];  // phi rho
      const T drho = sC[4];
      const T uu = ux * ux + uy * uy;
      const T eq_e = (T(2) * kappa - T(4) * phi) * drho + T(3) * m0 * uu;
      const T eq_ep = (T(4) * phi - T(3) * kappa) * drho - T(3) * m0 * uu;
      const T qfac = (kappa - T(2) * phi) * rho;  // phi rho (X - 2)
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
      const T pe = me - ph.s_e * (me - eq_e) + he * (S1 + Ca);
      const T pep = mep - ph.s_eps * (mep - eq_ep) - hep * S1;
      const T pqx = mqx - ph.s_q * (mqx - eq_qx) - hq * Fx;
      const T pqy = mqy - ph.s_q * (mqy - eq_qy) - hq * Fy;
      const T ppxx = mpxx - ph.s_nu * (mpxx - eq_pxx) + hn * (S7 + Cb);
      const T ppxy = mpxy - ph.s_nu * (mpxy - eq_pxy) + hn * (S8 + Cc);
      const T pm0 = sC[0];
      const T pjx = sC[1] + Fx;
      const T pjy = sC[2] + Fy;

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

      const int oo = yo * pitch + c;
      if (SHIFT) {
#pragma unroll
        for (int i = 0; i < 9; ++i) dst[i * P + oo] = static_cast<S>(o9[i] * ph.scale);
      } else {
        dst[0 * P + oo] = static_cast<S>(o9[0] + (phi * rho0 - ph.rest0_k));
#pragma unroll
        for (int i = 1; i < 5; ++i) dst[i * P + oo] = static_cast<S>(o9[i] + ph.rest_axis);
#pragma unroll
        for (int i = 5; i < 9; ++i) dst[i * P + oo] = static_cast<S>(o9[i] + ph.rest_diag);
      }
    }

#pragma unroll
    for (int i = 0; i < 9; ++i) { gC[i] = gB[i]; gB[i] = gA[i]; }
#pragma unroll
    for (int i = 0; i < 5; ++i) { sC[i] = sB[i]; sB[i] = sA[i]; }
#pragma unroll
    for (int i = 0; i < 4; ++i) bC[i] = bN[i];
  }
}

}  // namespace vanse_dev
