// step2_kernel.hpp -- two time steps of the plain MRTLB-VANSE step per pass
// over the populations in HBM.
//
// A workgroup of 2*NT lanes sweeps a strip of rows as the single-step kernel
// does, with two halves of NT lanes (whole waves) working on the same
// columns:
//   half 0 advances rows from t to t+1: pulls from HBM, moments, velocity,
//          collision -- and writes the post-collision deviations into an LDS
//          ring instead of HBM;
//   half 1 advances the same columns from t+1 to t+2 four rows behind: it
//          pulls from the LDS ring (the x and y shifts of streaming become
//          ring indices), and stores to HBM.
// The arithmetic of each half is that of the plain single step (Sec. 2.3:
// Eq. 7, 10, 13, 14-20, A1); only where the intermediate populations live
// differs, so HBM traffic per time step halves.  The intermediate state is
// kept as FP32 deviations from the rest state, which for FP32-shifted
// storage is exactly what the single step stores.
//
// Per iteration k each half runs three stages on rows yA = y0 - 5 - 4 half
// + k (A: moments), yA - 1 (B: velocity), yA - 2 (C: collision), with three
// workgroup barriers.  Half 0's collision row P feeds half 1's pull of row
// P - 1 one iteration later, and rows P - 2 and P - 3 two and three
// iterations later; the ring keeps three rows of each plane (four for the
// planes 2, 5, 6 pulled from below).
//
// Columns: lane t of either half is column x0 - 5 + t.  Half 0 forms moments
// on lanes [0, w+10), velocities on [1, w+9), collisions on [2, w+8); half 1
// on [3, w+7), [4, w+6), [5, w+5), the last being the strip's w <= NT - 10
// output columns.  Rows: the row block [y0, y1) is output by half 1; half 0
// covers y0 - 3 .. y1 + 2.
#pragma once

#include "step_kernel.hpp"

namespace vanse_dev {

template <typename T, int NT>
struct Step2Lds {
  T rho[2][3][NT];      // per half: delta-rho of the last three rows
  U4<T> u4[2][3][NT];   // per half: velocity data of the last three rows
  U2<T> u2[2][3][NT];
  T pop[30][NT];        // half 0's post-collision deviations (see pop_slot)
};

// Ring row of population plane i for the sweep-relative row index j >= 0:
// planes 0, 1, 3, 4, 7, 8 keep three rows, planes 2, 5, 6 four.
__device__ __forceinline__ int pop_slot(int i, int j) {
  constexpr int base[9] = {0, 3, 18, 6, 9, 22, 26, 12, 15};
  const bool deep = (i == 2 || i == 5 || i == 6);
  return base[i] + (deep ? (j & 3) : int(unsigned(j) % 3u));
}

template <typename S, typename T, bool SHIFT, bool WALLS, int NT>
__device__ __forceinline__ void step2_tile(const StepGeom& g, const StepPhys<T>& ph, int strip,
                                           int by, Step2Lds<T, NT>& L) {
  // uniform per wave (NT is a multiple of the wave size); read from the first
  // lane so that the compiler keeps everything derived from it -- rows, ring
  // slots, branches -- in scalar registers
  const int half = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / NT);
  const int t = int(threadIdx.x) - half * NT;
  const int nx = g.nx, ny = g.ny, pitch = g.pitch;
  const int x0 = strip * g.out_w;
  const int w = min(g.out_w, nx - x0);
  const int h = 3 * half;
  const bool live = t >= h && t < w + 10 - h;
  const bool ulane = t >= h + 1 && t < w + 9 - h;
  const bool olane = t >= h + 2 && t < w + 8 - h;
  const int c = wrap_index(x0 - 5 + t, nx);
  const int cm = (c == 0) ? nx - 1 : c - 1;
  const int cp = (c == nx - 1) ? 0 : c + 1;
  const int tl = max(t - 1, 0), tr = min(t + 1, NT - 1);
  constexpr unsigned SB = sizeof(S);
  constexpr unsigned TB = sizeof(T);

  T (*s_rho)[NT] = L.rho[half];
  U4<T> (*s_u4)[NT] = L.u4[half];
  U2<T> (*s_u2)[NT] = L.u2[half];

  const unsigned plane_bytes = unsigned(g.plane) * SB;
  const unsigned row_bytes = unsigned(pitch) * SB;
  const rsrc_t srcr = make_rsrc(g.src, 9u * plane_bytes);
  const rsrc_t dstr = make_rsrc(g.dst, 9u * plane_bytes);
  const rsrc_t phir = make_rsrc(g.phi, unsigned(g.plane) * TB);
  auto poff = [&](int i, int r) { return unsigned(i) * plane_bytes + unsigned(r) * row_bytes; };

  const int y0 = by * g.rows;
  const int y1 = min(y0 + g.rows, ny);
  const int nit = (y1 - y0) + 11;
  const int yoff = 5 + 4 * half;
  // sweep-relative row index (>= 0 for every row a ring holds) and the
  // three-row ring slot of the stage rings
  auto jr = [&](int y) { return y - y0 + 12; };
  auto s3 = [&](int y) { return int(unsigned(jr(y)) % 3u); };

  const T kappa = ph.kappa, rho0 = ph.rho0;
  const T third = T(1.0 / 3.0);
  const unsigned xcb = unsigned(c) * SB, xmb = unsigned(cm) * SB, xpb = unsigned(cp) * SB;
  const unsigned xcT = unsigned(c) * TB;

  // Loads of row yn: half 0 pulls the nine populations from HBM (rows
  // clamped inside walls, always in bounds) and phi; half 1 only needs phi.
  auto load_row = [&](int yn, RowIn<S, T>& in) {
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
    in.phi = bload<T>(phir, xcT, unsigned(r) * unsigned(pitch) * TB);
    if (half == 0) {
      S (&f)[9] = in.f;
      f[0] = bload<S>(srcr, xcb, poff(0, r));
      f[1] = bload<S>(srcr, xmb, poff(1, r));
      f[3] = bload<S>(srcr, xpb, poff(3, r));
      f[2] = bload<S>(srcr, xcb, bl ? poff(4, r) : poff(2, rs));
      f[5] = bload<S>(srcr, bl ? xcb : xmb, bl ? poff(7, r) : poff(5, rs));
      f[6] = bload<S>(srcr, bl ? xcb : xpb, bl ? poff(8, r) : poff(6, rs));
      f[4] = bload<S>(srcr, xcb, bh ? poff(2, r) : poff(4, rn));
      f[7] = bload<S>(srcr, bh ? xcb : xpb, bh ? poff(5, r) : poff(7, rn));
      f[8] = bload<S>(srcr, bh ? xcb : xmb, bh ? poff(6, r) : poff(8, rn));
    }
  };

  auto body = [&](int k, const RowIn<S, T>& in, RowState<T>& rA, const RowState<T>& rB,
                  const RowState<T>& rC, T (&bNew)[2], const T (&bOld)[2]) {
    const int yA = y0 - yoff + k;

    // ---------------- stage A: moments of row yA ----------------
    const bool rowA = (WALLS ? (yA >= 0 && yA < ny) : true) && (half == 0 || yA >= y0 - 2);
    if (rowA && live) {
      const T phi = in.phi;
      T q[9];
      if (half == 0) {
        if (SHIFT) {
#pragma unroll
          for (int i = 0; i < 9; ++i)
            q[i] = sizeof(S) == 2 ? static_cast<T>(in.f[i]) * ph.inv_scale : static_cast<T>(in.f[i]);
        } else {
          q[0] = static_cast<T>(in.f[0]) - (phi * rho0 - ph.rest0_k);
#pragma unroll
          for (int i = 1; i < 5; ++i) q[i] = static_cast<T>(in.f[i]) - ph.rest_axis;
#pragma unroll
          for (int i = 5; i < 9; ++i) q[i] = static_cast<T>(in.f[i]) - ph.rest_diag;
        }
      } else {
        // pull from half 0's ring: f_i(x) = f+_i(x - e_i), bounce-back at walls
        const bool bl = WALLS && yA == 0, bh = WALLS && yA == ny - 1;
        const int j0 = jr(yA), jm = j0 - 1, jp = j0 + 1;
        q[0] = L.pop[pop_slot(0, j0)][t];
        q[1] = L.pop[pop_slot(1, j0)][tl];
        q[3] = L.pop[pop_slot(3, j0)][tr];
        q[2] = bl ? L.pop[pop_slot(4, j0)][t] : L.pop[pop_slot(2, jm)][t];
        q[5] = bl ? L.pop[pop_slot(7, j0)][t] : L.pop[pop_slot(5, jm)][tl];
        q[6] = bl ? L.pop[pop_slot(8, j0)][t] : L.pop[pop_slot(6, jm)][tr];
        q[4] = bh ? L.pop[pop_slot(2, j0)][t] : L.pop[pop_slot(4, jp)][t];
        q[7] = bh ? L.pop[pop_slot(5, j0)][t] : L.pop[pop_slot(7, jp)][tr];
        q[8] = bh ? L.pop[pop_slot(6, j0)][t] : L.pop[pop_slot(8, jp)][tl];
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
      rA.drho = rA.dm0 * recip(phi);
      s_rho[s3(yA)][t] = rA.drho;
      // image below the lower wall; it shares its slot with row 2, written
      // two iterations later, after every stage that reads the image.  Above
      // the upper wall the image's slot would be row ny - 3's, still read, so
      // the stages read row ny - 1 itself there instead.
      if (WALLS && yA == 0) s_rho[s3(-1)][t] = rA.drho;
    }
    __syncthreads();

    // ---------------- stage B: velocity of row yA - 1 ----------------
    const int yb = yA - 1;
    const bool rowB = (WALLS ? (yb >= 0 && yb < ny) : true) && (yb >= y0 - 4 + 3 * half);
    if (rowB && ulane) {
      const int sc = s3(yb), ss = s3(yb - 1);
      const int sn = (WALLS && yb == ny - 1) ? sc : s3(yb + 1);  // image above the wall
      const T rE = s_rho[sc][tr], rW = s_rho[sc][tl];
      const T rN = s_rho[sn][t], rS = s_rho[ss][t];
      const T rNE = s_rho[sn][tr], rNW = s_rho[sn][tl];
      const T rSE = s_rho[ss][tr], rSW = s_rho[ss][tl];
      const T grx = stencil_dx(rE, rW, rNE, rSE, rNW, rSW);
      const T gry = stencil_dy(rN, rS, rNE, rNW, rSE, rSW);
      const T phi = rB.phi;
      const T kp = (kappa - phi) * third;
      const T sg = ph.scale_by_phi ? phi : T(1);
      const T Fx = kp * grx + sg * ph.gx;
      const T Fy = kp * gry + sg * ph.gy;
      const T m0 = phi * rho0 + rB.dm0;
      const T inv_m0 = recip(m0);
      const T ux = (rB.jx + T(0.5) * Fx) * inv_m0;
      const T uy = (rB.jy + T(0.5) * Fy) * inv_m0;
      const T rho = rho0 + rB.drho;
      U4<T> a;
      U2<T> b;
      a.ux = ux; a.uy = uy; a.mux = m0 * ux; a.rux = rho * ux;
      b.muy = m0 * uy; b.ruy = rho * uy;
      s_u4[s3(yb)][t] = a;
      s_u2[s3(yb)][t] = b;
      if (WALLS && yb == 0) {  // mirror image below the lower wall
        const int sg2 = s3(-1);
        U4<T> am;
        U2<T> bm;
        am.ux = -a.ux; am.uy = -a.uy; am.mux = -a.mux; am.rux = -a.rux;
        bm.muy = -b.muy; bm.ruy = -b.ruy;
        s_u4[sg2][t] = am;
        s_u2[sg2][t] = bm;
      }
      bNew[0] = Fx;
      bNew[1] = Fy;
    }
    __syncthreads();

    // ---------------- stage C: collide row yA - 2 ----------------
    const int yo = yA - 2;
    const bool rowC = (WALLS ? (yo >= 0 && yo < ny) : true) &&
                      (half == 0 ? (yo >= y0 - 3 && yo <= y1 + 2) : (yo >= y0 && yo < y1));
    if (rowC && olane) {
      // above the upper wall the image is row ny - 1 itself, velocities negated
      const bool top = WALLS && yo == ny - 1;
      const int uo = s3(yo), us = s3(yo - 1), un = top ? uo : s3(yo + 1);
      const U4<T> aC = s_u4[uo][t];
      const U4<T> aE = s_u4[uo][tr], aW = s_u4[uo][tl];
      U4<T> aN = s_u4[un][t];
      const U4<T> aS = s_u4[us][t];
      U4<T> aNE = s_u4[un][tr], aNW = s_u4[un][tl];
      const U4<T> aSE = s_u4[us][tr], aSW = s_u4[us][tl];
      U2<T> bN = s_u2[un][t];
      const U2<T> bS = s_u2[us][t];
      U2<T> bNE = s_u2[un][tr], bNW = s_u2[un][tl];
      const U2<T> bSE = s_u2[us][tr], bSW = s_u2[us][tl];
      if (top) {
        auto neg4 = [](U4<T>& v) { v.ux = -v.ux; v.uy = -v.uy; v.mux = -v.mux; v.rux = -v.rux; };
        auto neg2 = [](U2<T>& v) { v.muy = -v.muy; v.ruy = -v.ruy; };
        neg4(aN); neg4(aNE); neg4(aNW);
        neg2(bN); neg2(bNE); neg2(bNW);
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
      const T kmp = kappa - phi;
      const T ux = aC.ux, uy = aC.uy, Fx = bOld[0], Fy = bOld[1];

      // penalty source (Eq. 20), static void fraction
      const T Ca = -kappa * (d_rux_x + d_ruy_y) + T(2) * kmp * rho * (d_ux_x + d_uy_y) +
                   (T(3) - T(2) * X) * (d_mux_x + d_muy_y);
      const T Cb = -kappa * (d_rux_x - d_ruy_y) + T(2.0 / 3.0) * kmp * rho * (d_ux_x - d_uy_y) +
                   (d_mux_x - d_muy_y);
      const T Cc = third * kmp * rho * (d_uy_x + d_ux_y);

      // equilibria (Eq. 18) minus those of the rest state
      const T m0 = phi * rho0 + rC.dm0;
      const T drho = rC.drho;
      const T uu = ux * ux + uy * uy;
      const T eq_e = (T(2) * kappa - T(4) * phi) * drho + T(3) * m0 * uu;
      const T eq_ep = (T(4) * phi - T(3) * kappa) * drho - T(3) * m0 * uu;
      const T qfac = (kappa - T(2) * phi) * rho;
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

      if (half == 0) {  // into the ring for the second step
        const int jo = jr(yo);
#pragma unroll
        for (int i = 0; i < 9; ++i) L.pop[pop_slot(i, jo)][t] = o9[i];
      } else if (SHIFT) {
#pragma unroll
        for (int i = 0; i < 9; ++i)
          bstore(static_cast<S>(sizeof(S) == 2 ? o9[i] * ph.scale : o9[i]), dstr, xcb, poff(i, yo));
      } else {
        bstore(static_cast<S>(o9[0] + (phi * rho0 - ph.rest0_k)), dstr, xcb, poff(0, yo));
#pragma unroll
        for (int i = 1; i < 5; ++i) bstore(static_cast<S>(o9[i] + ph.rest_axis), dstr, xcb, poff(i, yo));
#pragma unroll
        for (int i = 5; i < 9; ++i) bstore(static_cast<S>(o9[i] + ph.rest_diag), dstr, xcb, poff(i, yo));
      }
    }
    // the ring rows written here are pulled in the next iteration
    __syncthreads();
  };

  // Software pipeline as in the single step: the loads of row yA + 1 are in
  // flight while row yA is processed; unrolled by six (a multiple of the
  // three-row period of the states) so nothing is copied.
  RowState<T> R0{}, R1{}, R2{};
  T b0[2] = {0, 0}, b1[2] = {0, 0};
  RowIn<S, T> ia{}, ib{};
  load_row(y0 - yoff, ia);
  for (int k = 0; k < nit; k += 6) {
    load_row(y0 - yoff + 1 + k, ib);
    body(k + 0, ia, R0, R2, R1, b0, b1);
    if (k + 1 >= nit) break;
    load_row(y0 - yoff + 2 + k, ia);
    body(k + 1, ib, R1, R0, R2, b1, b0);
    if (k + 2 >= nit) break;
    load_row(y0 - yoff + 3 + k, ib);
    body(k + 2, ia, R2, R1, R0, b0, b1);
    if (k + 3 >= nit) break;
    load_row(y0 - yoff + 4 + k, ia);
    body(k + 3, ib, R0, R2, R1, b1, b0);
    if (k + 4 >= nit) break;
    load_row(y0 - yoff + 5 + k, ib);
    body(k + 4, ia, R1, R0, R2, b0, b1);
    if (k + 5 >= nit) break;
    load_row(y0 - yoff + 6 + k, ia);
    body(k + 5, ib, R2, R1, R0, b1, b0);
  }
}

// Two time steps per launch: workgroup b takes strip b % strips, row block
// b / strips; 2 NT lanes (two halves of NT), four waves per SIMD.
template <typename S, typename T, bool SHIFT, bool WALLS, int NT>
__global__ void __launch_bounds__(2 * NT) __attribute__((amdgpu_waves_per_eu(4)))
vanse_step2_kernel(StepGeom g, StepPhys<T> ph) {
  __shared__ Step2Lds<T, NT> lds;
  step2_tile<S, T, SHIFT, WALLS, NT>(g, ph, int(blockIdx.x) % g.strips, int(blockIdx.x) / g.strips,
                                     lds);
}

}  // namespace vanse_dev
