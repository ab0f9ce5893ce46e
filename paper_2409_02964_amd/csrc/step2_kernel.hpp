// step2_kernel.hpp -- two time steps of the plain MRTLB-VANSE step per pass
// over the populations in HBM.
//
// A workgroup of 2*NT lanes sweeps a strip of rows as the single-step kernel
// does, with two halves of NT lanes (whole waves) working on the same
// columns:
//   half 0 advances rows from t to t+1: pulls from HBM, moments, velocity,
//          collision -- and writes the post-collision deviations into an LDS
//          ring instead of HBM;
//   half 1 advances the same columns from t+1 to t+2 five rows behind: it
//          pulls from the LDS ring (the x and y shifts of streaming become
//          ring indices), and stores to HBM.
// Each half computes the plain single step's scheme (Sec. 2.3: Eq. 7, 10,
// 13, 14-20, A1), with the Eq. (10) sums in the separable form below; the
// intermediate populations never reach HBM, so HBM traffic per time step
// halves.  The intermediate state is kept as deviations from the rest state
// in the arithmetic type: with FP32 arithmetic the format the single step
// stores with FP32-shifted storage; FP64 keeps it in FP64 (halves of 128
// lanes then, as the rings take twice the bytes per lane).
//
// Per iteration k each half runs three stages on rows yA = y0 - 5 - 5 half
// + k (A: moments), yA - 1 (B: velocity), yA - 2 (C: collision), with two
// workgroup barriers (after stages A and B).  Half 0's collision row P feeds
// half 1's pull of row P - 1 two iterations later, and rows P - 2 and P - 3
// three and four iterations later; the ring keeps four rows of each plane,
// row P taking the slot of row P - 4 after half 1's last read of it (see the
// end of the sweep iteration).  Half-way
// bounce-back at a wall enters half 1's pull through image rows of the ring
// (row -1 of planes 2, 5, 6 and row ny of planes 4, 7, 8), which half 0
// fills from the wall row once per sweep, so the pull itself never tests
// for walls.
//
// Half 0's pulls from HBM: each row is loaded straight into LDS (buffer
// loads with the LDS destination) two rows ahead, into a two-slot staging
// area, so the loads in flight hold no registers and have two iterations to
// land.  Half 1 issues no loads: phi (and beta) of a row reach it through
// the population ring with the row.
//
// The Eq. (10) derivatives use the stencil's separable form.  With
//   D(y) = g(x+1, y) - g(x-1, y),   S(y) = g(x+1, y) + g(x-1, y) + 4 g(x, y)
// for a field g on row y, the stencil is
//   12 d_x g(y) = 4 D(y) + D(y-1) + D(y+1),   12 d_y g(y) = S(y+1) - S(y-1).
// A lane sweeps one column, so each row's D and S are formed once, from the
// row's own values and its two neighbours in LDS, and the two rows below stay
// in registers.  The LDS rings of delta-rho and of the velocity data then
// hold a single row.  The rows beyond a wall (the centre-value image of
// delta-rho, the negated image of the velocity fields) are written into
// those rings above the upper wall and formed in registers from the D and S
// of row 0 below the lower wall.
//
// Solid nodes (FEAT_MASK; the uint16 flags of the single step: bit 0 the
// node is solid, bit i its neighbour x + e_i is):
//   - Half-way bounce-back: a fluid node pulls f_i from its own slot opp(i)
//     when bit opp(i) is set.  Half 0's staged row then takes per-lane
//     offsets, so the flags of a row must be known when its loads are
//     issued: each staged row also carries the flags of the row two ahead,
//     which the sweep keeps in registers until that row is staged.  Half 1
//     takes the own-slot value from the ring (the flags ride with the row).
//   - Eq. (10): a solid neighbour stands in with the centre value (negated
//     for the velocity-like fields).  Solid nodes write zeros into the
//     single-row rings, so the separable sums leave them out, and the centre
//     value times Kx = sum of c_i e_ix over the flagged neighbours (c_i = 4
//     on the axes, 1 on the diagonals; Ky alike) restores the stand-ins.
//   - Solid nodes keep the rest state (zero deviations).
//
// A moving phi (FEAT_DYNPHI; the d_t phi term of Eq. 20): half 0 stages
// phi(t), phi(t+1) and phi(t+2) (and, with the drag, both steps' beta) with
// each row, and writes the second step's phi and beta into the ring as soon
// as the row has landed; half 1 takes its d_t phi from there.  The ring and
// shifted storage hold deviations from the rest state of the phi of the next
// pull.
//
// The scheme variants (Sec. 2.3 and Appendix B), also with solid nodes:
// model B (FEAT_SCHEME here) takes kappa - 1 for kappa - phi in F^p and the
// source term, the solid-neighbour terms included; the Appendix B
// equilibrium (FEAT_EQ2) its q moments and the penalty of Eq. (B3), whose
// four extra derivatives come from the same velocity records (their D and S
// carried as the others are, their solid-neighbour terms gathered with the
// others').
//
// Half 0 issues its staging loads after the first barrier; with FP16
// storage (bound by the pipeline rather than HBM) those of the rows below
// and above follow the second barrier, in the longer phase.
//
// Columns: lane t of either half is column x0 - 5 + t.  Half 0 forms moments
// on lanes [0, w+10), velocities on [1, w+9), collisions on [2, w+8); half 1
// on [3, w+7), [4, w+6), [5, w+5), the last being the strip's w <= NT - 10
// output columns.  Rows: the row block [y0, y1) is output by half 1; half 0
// covers y0 - 3 .. y1 + 2.
#pragma once

#include <stdint.h>

#include "step_kernel.hpp"

namespace vanse_dev {

// NP: planes of the population ring -- the nine populations, phi and, with
// the linear drag, its coefficient beta, and with solid nodes their flags
template <typename T, int NT, int NP>
struct Step2Lds {
  T rho[2][NT];      // per half: delta-rho of the row of stage A (read by B)
  U4<T> u4[2][NT];   // per half: velocity data of the row of stage B (read by C)
  U2<T> u2[2][NT];
  T pop[4 * NP][NT];  // half 0's post-collision deviations, phi, beta (see pop_slot)
};

// Half 0's staging of a pulled row: the nine populations, phi, (with the
// drag) beta and (with solid nodes, last) the flags of the row two ahead, as
// NW rows of 4-byte words, each lane's word at its own
// position.  A 2-byte load with LDS destination fills its lane's word,
// zero-extended; an 8-byte value takes two words, its low half in row 2i
// and its high half in row 2i + 1.  Two slots, each its own LDS object,
// passed to the tile as distinct restrict pointers: the compiler then orders
// a read of one slot after the loads into that slot only, not after the
// loads of the row ahead in flight into the other.
template <int NT, int NW>
struct Step2Stage {
  float v[NW][NT];
};

// Wait until at most n vector-memory operations of this wave are
// outstanding (s_waitcnt with expcnt and lgkmcnt left at their maximum).
// The compiler does not order LDS reads after loads into LDS by itself, so
// the asm statement keeps the reads that follow below the wait.
template <int n>
__device__ __forceinline__ void wait_vm() {
  static_assert(n >= 0 && n < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14));
  __asm__ volatile("" ::: "memory");
}

// Workgroup barrier for LDS traffic: this wave's LDS reads and writes
// complete, then s_barrier.  Unlike __syncthreads() it does not wait for the
// wave's loads into LDS (the staging of rows ahead), which wait_vm orders
// before their readers.
__device__ __forceinline__ void lds_barrier() {
  __asm__ volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (0 << 8) | (3 << 14));  // lgkmcnt(0)
  __builtin_amdgcn_s_barrier();
  __asm__ volatile("" ::: "memory");
}

// LDS-qualified object type
template <typename X>
using lds_t = __attribute__((address_space(3))) X;

// The address of an LDS object as a value the compiler cannot trace back to
// the object.  The tile takes its three LDS objects as restrict pointers made
// this way; inlining then tags every LDS access with the object it belongs
// to, which lets the compiler order a read of one staging slot after the
// loads into that slot only (a read it cannot attribute waits for every load
// into LDS in flight, the row ahead included).
template <typename X>
__device__ __forceinline__ lds_t<X>* lds_handle(X* p) {
  unsigned u = unsigned(uintptr_t((lds_t<X>*)p));
  __asm__ volatile("" : "+s"(u));
  return (lds_t<X>*)uintptr_t(u);
}

// Member-wise copies of the velocity records to and from LDS (the implicit
// copy operations take generic-address-space objects)
template <typename T>
__device__ __forceinline__ U4<T> lds_get(const lds_t<U4<T>>& v) {
  U4<T> r;
  r.ux = v.ux; r.uy = v.uy; r.mux = v.mux; r.rux = v.rux;
  return r;
}
template <typename T>
__device__ __forceinline__ U2<T> lds_get(const lds_t<U2<T>>& v) {
  U2<T> r;
  r.muy = v.muy; r.ruy = v.ruy;
  return r;
}
template <typename T>
__device__ __forceinline__ void lds_put(lds_t<U4<T>>& d, const U4<T>& v) {
  d.ux = v.ux; d.uy = v.uy; d.mux = v.mux; d.rux = v.rux;
}
template <typename T>
__device__ __forceinline__ void lds_put(lds_t<U2<T>>& d, const U2<T>& v) {
  d.muy = v.muy; d.ruy = v.ruy;
}

// Value i of a staged row (type X: 8, 4 or 2 bytes) on lane t
template <typename X, int NT, int NW>
__device__ __forceinline__ X staged(const lds_t<Step2Stage<NT, NW>>* st, int i, int t) {
  if constexpr (sizeof(X) == 8) {
    const unsigned long long lo = __builtin_bit_cast(unsigned, float(st->v[2 * i][t]));
    const unsigned long long hi = __builtin_bit_cast(unsigned, float(st->v[2 * i + 1][t]));
    return __builtin_bit_cast(X, lo | (hi << 32));
  } else if constexpr (sizeof(X) == 4) {
    return __builtin_bit_cast(X, float(st->v[i][t]));
  } else {
    return __builtin_bit_cast(X, (unsigned short)__builtin_bit_cast(unsigned, float(st->v[i][t])));
  }
}

// D and S (see above) of delta-rho on one row
template <typename T>
struct RhoDS {
  T d, s;
};

// D of the fields differentiated in x and S of those differentiated in y by
// the penalty of Eq. (20) on one row, and the node's velocity
template <typename T>
struct VelDS {
  T d_rux, d_ux, d_uy, d_mux;
  T s_ruy, s_uy, s_ux, s_muy;
  T ux, uy;
  // the Appendix B penalty's four more: D of rho u_y and phi rho u_y, S of
  // rho u_x and phi rho u_x (formed only there)
  T d_ruy, d_muy, s_rux, s_mux;
};

// the image row beyond a wall: velocity-like fields negated
template <typename T>
__device__ __forceinline__ VelDS<T> mirrored(const VelDS<T>& v) {
  VelDS<T> r;
  r.d_rux = -v.d_rux; r.d_ux = -v.d_ux; r.d_uy = -v.d_uy; r.d_mux = -v.d_mux;
  r.s_ruy = -v.s_ruy; r.s_uy = -v.s_uy; r.s_ux = -v.s_ux; r.s_muy = -v.s_muy;
  r.ux = -v.ux; r.uy = -v.uy;
  r.d_ruy = -v.d_ruy; r.d_muy = -v.d_muy; r.s_rux = -v.s_rux; r.s_mux = -v.s_mux;
  return r;
}

// Ring row of population plane i (after the nine populations: phi, beta,
// phi(t+2) and the solid flags, see step2_planes) for the sweep-relative row
// index j >= 0
__device__ __forceinline__ int pop_slot(int i, int j) { return 4 * i + (j & 3); }

// Planes a row carries to half 1: nine populations and phi of its step,
// plus beta with the drag, phi(t+2) with a moving phi and the solid flags
// with a mask (in this order)
template <int FEAT>
constexpr int step2_planes() {
  return 10 + ((FEAT & FEAT_DRAG) ? 1 : 0) + ((FEAT & FEAT_DYNPHI) ? 1 : 0) + ((FEAT & FEAT_MASK) ? 1 : 0);
}

// Values of a staged row: nine populations, phi and beta (with the drag) of
// the first step, and with a moving phi phi(t+1), phi(t+2) and the second
// step's beta (with the drag)
template <int FEAT>
constexpr int step2_values() {
  constexpr int D = (FEAT & FEAT_DRAG) ? 1 : 0;
  return 10 + D + ((FEAT & FEAT_DYNPHI) ? 2 + D : 0);
}

// 4-byte words of a staged row: one per value, two for 8-byte values; the
// flags (of the row two ahead) take one
template <typename S, int FEAT>
constexpr int step2_words() {
  return step2_values<FEAT>() * (sizeof(S) == 8 ? 2 : 1) + ((FEAT & FEAT_MASK) ? 1 : 0);
}

// The variants whose extra planes take so much LDS, or extra carried sums so
// many registers, that their halves are narrower (solid nodes with the drag;
// a moving phi; the Appendix B penalty)
constexpr bool step2_wide_rows(int feat) {
  return ((feat & FEAT_MASK) && (feat & FEAT_DRAG)) || (feat & FEAT_DYNPHI) || (feat & FEAT_EQ2);
}

// Waves per SIMD of the two-step kernels: four in FP32 arithmetic (128
// registers), two in FP64 (256); three for the narrow-half variants in FP32
// (168: at 128 they would spill, and a spill reloaded in the sweep waits for
// the row staged ahead as well)
constexpr int step2_waves_of(int tbytes, int feat) { return tbytes == 8 ? 2 : (step2_wide_rows(feat) ? 3 : 4); }
template <typename T, int FEAT>
constexpr int step2_waves() { return step2_waves_of(int(sizeof(T)), FEAT); }

// Lanes per half: 256 in FP32 arithmetic and 128 in FP64 (whose rings take
// twice the bytes per lane); half that for the variants with wide rows
// (three workgroups per CU in FP32).
constexpr int step2_nt_of(int tbytes, int feat) {
  return (tbytes == 8 ? 128 : 256) >> (step2_wide_rows(feat) ? 1 : 0);
}

// LDS bytes of one two-step workgroup
template <typename S, typename T, int FEAT, int NT>
constexpr unsigned step2_lds_bytes() {
  return unsigned(sizeof(Step2Lds<T, NT, step2_planes<FEAT>()>) + 2 * sizeof(Step2Stage<NT, step2_words<S, FEAT>()>));
}

// Flagged-neighbour sums of the Eq. (10) stencils: sum over the neighbours
// flagged in nb (bits 1..8) of c_i e_ix and c_i e_iy, with c_i = 4 on the
// axes and 1 on the diagonals (each 12 times the stencil's weight)
__device__ __forceinline__ int solid_kx(unsigned nb) {
  const int b = int(nb);
  return 4 * (((b >> 1) & 1) - ((b >> 3) & 1)) + ((((b >> 5) & 1) + ((b >> 8) & 1)) - (((b >> 6) & 1) + ((b >> 7) & 1)));
}
__device__ __forceinline__ int solid_ky(unsigned nb) {
  const int b = int(nb);
  return 4 * (((b >> 2) & 1) - ((b >> 4) & 1)) + ((((b >> 5) & 1) + ((b >> 6) & 1)) - (((b >> 7) & 1) + ((b >> 8) & 1)));
}

// Solid flags of the rows in flight (see the sweep)
struct FlagRows {
  unsigned lo, hi;
};

// A moving phi: the second step's phi(t+1), phi(t+2) and beta of the row
// staged one iteration before
template <typename T>
struct DynRow {
  T phi1, phi2, beta2;
};

// true on every lane if any lane of the wave has cond
__device__ __forceinline__ bool wave_any(bool cond) { return __builtin_amdgcn_ballot_w64(cond) != 0; }

// The solid flags as a value of the ring's type and back (bit copies)
template <typename T>
__device__ __forceinline__ T flags_as(unsigned nb) {
  if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, (unsigned long long)nb);
  else return __builtin_bit_cast(T, nb);
}
template <typename T>
__device__ __forceinline__ unsigned flags_of(T v) {
  if constexpr (sizeof(T) == 8) return unsigned(__builtin_bit_cast(unsigned long long, v));
  else return __builtin_bit_cast(unsigned, v);
}

// FEAT: the plain step plus any of FEAT_FORCE (a per-node force field added
// to F^B), FEAT_DRAG (the linear drag, u solved in closed form as in the
// single step), and FEAT_MASK (solid nodes; no walls in x) or FEAT_DYNPHI
// (a moving phi) or FEAT_SCHEME (model B alone) or FEAT_EQ2 (the Appendix B
// equilibrium).  Absent force, drag and flag planes read as zero.
template <typename S, typename T, bool SHIFT, bool WALLS, int FEAT, int NT>
__device__ inline void step2_tile(
    const StepGeom& g, const StepPhys<T>& ph, int strip, int by,
    lds_t<Step2Lds<T, NT, step2_planes<FEAT>()>>* __restrict__ Lp,
    lds_t<Step2Stage<NT, step2_words<S, FEAT>()>>* __restrict__ st0,
    lds_t<Step2Stage<NT, step2_words<S, FEAT>()>>* __restrict__ st1) {
  static_assert((FEAT & ~(FEAT_FORCE | FEAT_DRAG | FEAT_MASK | FEAT_DYNPHI | FEAT_SCHEME | FEAT_EQ2)) == 0,
                "force field, linear drag, solid nodes, a moving phi, model B and Appendix B only");
  static_assert(!((FEAT & FEAT_EQ2) && (FEAT & (FEAT_DYNPHI | FEAT_SCHEME))),
                "the Appendix B equilibrium without a moving phi");
  static_assert(!((FEAT & FEAT_MASK) && (FEAT & FEAT_DYNPHI)), "solid nodes or a moving phi");
  static_assert(!((FEAT & FEAT_SCHEME) && (FEAT & FEAT_DYNPHI)), "model B without a moving phi");
  constexpr bool DRAG = (FEAT & FEAT_DRAG) != 0;
  constexpr bool FORCE = (FEAT & FEAT_FORCE) != 0;
  constexpr bool MASK = (FEAT & FEAT_MASK) != 0;
  constexpr bool DYN = (FEAT & FEAT_DYNPHI) != 0;
  // FEAT_SCHEME here is model B alone (Sec. 2.3): kappa - 1 in place of
  // kappa - phi in F^p (Eq. 13) and in the kappa - phi factors of Eq. (20)
  constexpr bool MODEL_B = (FEAT & FEAT_SCHEME) != 0;
  // FEAT_EQ2: the Appendix B equilibrium (B2 moments, the twelve-derivative
  // penalty of Eq. B3), model B then a run-time flag
  constexpr bool EQ2 = (FEAT & FEAT_EQ2) != 0;
  const bool kappa_less_one = MODEL_B || (EQ2 && ph.model_b != 0);
  // ring planes after the populations and phi, and staged values after the
  // populations, phi and beta (see step2_planes and step2_values)
  constexpr int PL_PHIN2 = DRAG ? 11 : 10;               // phi(t+2)
  constexpr int PL_NB = DRAG ? 11 : 10;                  // the solid flags
  constexpr int V_PHIN = DRAG ? 11 : 10, V_PHIN2 = V_PHIN + 1, V_BETA2 = V_PHIN + 2;
  constexpr int NW = step2_words<S, FEAT>();
  constexpr unsigned BOUNCE = 0x1FEu;                    // neighbour bits of the flags
  auto& L = *Lp;
  static_assert(((sizeof(S) == 4 || sizeof(S) == 2) && sizeof(T) == 4) ||
                    (sizeof(S) == 8 && sizeof(T) == 8),
                "4- or 2-byte storage with FP32 arithmetic, or FP64 throughout");
  // uniform per wave (NT is a multiple of the wave size); read from the first
  // lane so that the compiler keeps everything derived from it -- rows, ring
  // slots, branches -- in scalar registers
  const int half = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / NT);
  // Wave priorities (s_setprio: the order in which a SIMD issues the
  // instructions of its waves; the results do not change).  With FP32
  // storage and halves of 256 lanes half 1's waves go first throughout, then
  // half 0's waves between the start of a row and its second barrier (stages
  // A and B, the short phase), then half 0's waves in stage C.  Otherwise
  // (FP16 or FP64 storage, or halves narrower than 256 lanes: batches and
  // the FP32 variants with wide rows) only the phase counts: stages A and B
  // of either half before stage C (FP16 storage issues its staging loads of
  // the shifted rows after the second barrier).
  // Measured against no priorities on the 4096^2 channel: 146 -> 136.5 us
  // per step in FP32-shifted storage, 113 -> 109 in FP16-shifted storage,
  // 328 -> 314 in FP64; on the 256-lattice FP32 batch with 128-lane halves
  // the phase order gains 1% over the three levels.  The orders tried
  // besides (half 0 first, the phase order alone with 256-lane FP32 halves,
  // half 1 first with FP16 or FP64 storage, ...) gained less or lost.
  constexpr bool PRIO_PHASE = sizeof(S) != 4 || NT < 256;        // both halves, by phase
  constexpr bool PRIO_HALF0_PHASE = sizeof(S) == 4 && NT >= 256;  // half 0 by phase, under half 1
  if (!PRIO_PHASE && half == 1) __builtin_amdgcn_s_setprio(2);
  const int t = int(threadIdx.x) - half * NT;
  const int nx = g.nx, ny = g.ny, pitch = g.pitch;
  // Half 1 runs LAG = 5 rows behind half 0 (see the end of the body)
  constexpr int LAG = 5;
  const int yoff = 5 + LAG * half;
  const int x0 = strip * g.out_w;
  const int w = min(g.out_w, nx - x0);
  const int h = 3 * half;
  // Lanes whose moments, velocities and collisions are valid: [h, w+10-h),
  // [h+1, w+9-h) and [h+2, w+8-h).  Only the collision's stores are masked;
  // moments, velocities, D and S are formed on every lane (all loads stay in
  // bounds), so the state carried from row to row is never written under a
  // lane mask, which would cost a copy of each carried value per row.
  // Values of the other lanes are never used.
  const bool olane = t >= h + 2 && t < w + 8 - h;
  auto* s_rho = L.rho[half];
  auto* s_u4 = L.u4[half];
  auto* s_u2 = L.u2[half];
  const int c = wrap_index(x0 - 5 + t, nx);
  const int cm = (c == 0) ? nx - 1 : c - 1;
  const int cp = (c == nx - 1) ? 0 : c + 1;
  const int tl = max(t - 1, 0), tr = min(t + 1, NT - 1);
  constexpr unsigned SB = sizeof(S);
  constexpr unsigned TB = sizeof(T);


  const unsigned plane_bytes = unsigned(g.plane) * SB;
  const unsigned row_bytes = unsigned(pitch) * SB;
  const rsrc_t srcr = make_rsrc(g.src, 9u * plane_bytes);
  const rsrc_t dstr = make_rsrc(g.dst, 9u * plane_bytes);
  const rsrc_t phir = make_rsrc(g.phi, unsigned(g.plane) * TB);
  const rsrc_t betar = make_rsrc(g.beta, (DRAG && g.beta) ? unsigned(g.plane) * TB : 0u);
  const rsrc_t fxr = make_rsrc(g.fxf, (FORCE && g.fxf) ? unsigned(g.plane) * TB : 0u);
  const rsrc_t fyr = make_rsrc(g.fyf, (FORCE && g.fyf) ? unsigned(g.plane) * TB : 0u);
  // a moving phi: phi(t+1) and the second step's phi(t+2), beta and force
  const rsrc_t phinr = make_rsrc(g.phin, DYN ? unsigned(g.plane) * TB : 0u);
  const rsrc_t phin2r = make_rsrc(g.phin2, DYN ? unsigned(g.plane) * TB : 0u);
  const rsrc_t beta2r = make_rsrc(g.beta2, (DYN && DRAG && g.beta2) ? unsigned(g.plane) * TB : 0u);
  const rsrc_t fx2r = make_rsrc(g.fxf2, (DYN && FORCE && g.fxf2) ? unsigned(g.plane) * TB : 0u);
  const rsrc_t fy2r = make_rsrc(g.fyf2, (DYN && FORCE && g.fyf2) ? unsigned(g.plane) * TB : 0u);
  const rsrc_t nbrr = make_rsrc(g.nbr, (MASK && g.nbr) ? unsigned(g.plane) * 2u : 0u);
  auto poff = [&](int i, int r) { return unsigned(i) * plane_bytes + unsigned(r) * row_bytes; };
  // row of the flags a staged row yn carries (those of row yn + 2)
  auto flag_row = [&](int yn) {
    return unsigned(WALLS ? min(max(yn + 2, 0), ny - 1) : wrap_index(yn + 2, ny)) * unsigned(pitch) * 2u;
  };

  const int y0 = by * g.rows;
  const int y1 = min(y0 + g.rows, ny);
  const int nit = (y1 - y0) + 7 + LAG;
  // sweep-relative row index of the population ring (>= 0 for every row it
  // holds)
  auto jr = [&](int y) { return y - y0 + 12; };

  const T kappa = ph.kappa, rho0 = ph.rho0;
  const unsigned xcb = unsigned(c) * SB, xmb = unsigned(cm) * SB, xpb = unsigned(cp) * SB;
  const unsigned xcT = unsigned(c) * TB;

  // The pull of row yn from HBM: ld(i, buffer, lane offset, row offset) for
  // the nine populations (i = 0..8), phi (i = 9), beta (i = 10), the moving
  // phi's values (V_PHIN, V_PHIN2, V_BETA2) and the flags of row yn + 2
  // (i = -1).  Rows are clamped inside walls, so every load is in bounds.
  // fl: the flags of row yn.
  // part: 0 every load; 1 phi and the other node values, the flags and the
  // populations of the row itself (0, 1, 3); 2 those of the rows below and
  // above (2, 5, 6, 4, 7, 8)
  auto pull_row = [&](int yn, unsigned fl, auto&& ld, int part = 0) {
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
    if (part != 2) {
      ld(9, phir, xcT, unsigned(r) * unsigned(pitch) * TB);
      if (DRAG) ld(10, betar, xcT, unsigned(r) * unsigned(pitch) * TB);
      if (DYN) {
        ld(V_PHIN, phinr, xcT, unsigned(r) * unsigned(pitch) * TB);
        ld(V_PHIN2, phin2r, xcT, unsigned(r) * unsigned(pitch) * TB);
        if (DRAG) ld(V_BETA2, beta2r, xcT, unsigned(r) * unsigned(pitch) * TB);
      }
      if (MASK) ld(-1, nbrr, unsigned(c) * 2u, flag_row(yn));
      ld(0, srcr, xcb, poff(0, r));
    }
    if (MASK && wave_any((fl & BOUNCE) != 0)) {
      // a wave next to a solid node: per lane the pulled slot, or the own
      // node's opposite slot when the source is solid (whole byte offsets
      // in the per-lane operand); wall rows as below
      auto pick = [&](int i, unsigned vcol, unsigned soff, int opp) {
        // the uniform parts kept opaque: folded into the per-lane columns
        // they would become loop-invariant registers
        unsigned so = poff(opp, r), sp = soff;
        __asm__ volatile("" : "+s"(so), "+s"(sp));
        ld(i, srcr, solid_bit(fl, opp) ? so + xcb : sp + vcol, 0u);
      };
      pick(1, xmb, poff(1, r), 3);
      pick(3, xpb, poff(3, r), 1);
      pick(2, xcb, bl ? poff(4, r) : poff(2, rs), 4);
      pick(5, bl ? xcb : xmb, bl ? poff(7, r) : poff(5, rs), 7);
      pick(6, bl ? xcb : xpb, bl ? poff(8, r) : poff(6, rs), 8);
      pick(4, xcb, bh ? poff(2, r) : poff(4, rn), 2);
      pick(7, bh ? xcb : xpb, bh ? poff(5, r) : poff(7, rn), 5);
      pick(8, bh ? xcb : xmb, bh ? poff(6, r) : poff(8, rn), 6);
      return;
    }
    if (part != 2) {
      ld(1, srcr, xmb, poff(1, r));
      ld(3, srcr, xpb, poff(3, r));
    }
    if (part == 1) return;
    if (WALLS && (bl || bh)) {
      // a wall row (taken on two rows per sweep, so the others need no
      // per-lane selects of their column offsets)
      ld(2, srcr, xcb, bl ? poff(4, r) : poff(2, rs));
      ld(5, srcr, bl ? xcb : xmb, bl ? poff(7, r) : poff(5, rs));
      ld(6, srcr, bl ? xcb : xpb, bl ? poff(8, r) : poff(6, rs));
      ld(4, srcr, xcb, bh ? poff(2, r) : poff(4, rn));
      ld(7, srcr, bh ? xcb : xpb, bh ? poff(5, r) : poff(7, rn));
      ld(8, srcr, bh ? xcb : xmb, bh ? poff(6, r) : poff(8, rn));
    } else {
      ld(2, srcr, xcb, poff(2, rs));
      ld(5, srcr, xmb, poff(5, rs));
      ld(6, srcr, xpb, poff(6, rs));
      ld(4, srcr, xcb, poff(4, rn));
      ld(7, srcr, xpb, poff(7, rn));
      ld(8, srcr, xmb, poff(8, rn));
    }
  };
  // Half 0's loads of row yn into staging slot sl; each wave's 64 lanes
  // fill 64 consecutive words from the wave's base.
  const int wb = __builtin_amdgcn_readfirstlane(t & ~63);
  auto stage_row = [&](int yn, int sl, unsigned fl, int part = 0) {
    pull_row(yn, fl, [&](int i, rsrc_t rs, unsigned v, unsigned so) {
      auto* st = sl ? st1 : st0;
      if (i < 0) {  // the flags of row yn + 2: the last word
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_t<void>*)&st->v[NW - 1][wb], 2, v, so, 0, 0);
        return;
      }
      if constexpr (sizeof(S) == 8) {
        // low and high words (phi and beta are FP64 too); the high word's 4
        // bytes go into the uniform offset: an immediate offset would move
        // the LDS destination as well
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_t<void>*)&st->v[2 * i][wb], 4, v, so, 0, 0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_t<void>*)&st->v[2 * i + 1][wb], 4, v, so + 4u, 0, 0);
      } else {
        auto* d = (lds_t<void>*)&st->v[i][wb];
        if (i >= 9 || sizeof(S) == 4) __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, d, 4, v, so, 0, 0);
        else __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, d, 2, v, so, 0, 0);
      }
    }, part);
  };

  // D and S of the two rows below the one that stage B (rm, rc) and stage C
  // (vm, vc) read from LDS
  RhoDS<T> rm{}, rc{};
  VelDS<T> vm{}, vc{};

  // One sweep iteration.  Rows beyond a wall: above the upper wall stage A
  // and stage B write the image of row ny - 1 into the single-row rings;
  // below the lower wall the image of row 0 replaces the carried D and S of
  // row -1 before the stage that needs it.
  // With solid nodes the flags of the rows in flight sit in 10-bit fields of
  // two registers, shifted by one field per iteration: fl.hi holds those of
  // rows yA, yA - 1 and yA - 2 (stages A, B and C), and half 0's fl.lo those
  // of rows yA + 2 and yA + 1 (staged with row yA and yA - 1).
  auto body = [&](int k, int sl, RowState<T>& rA, const RowState<T>& rB,
                  const RowState<T>& rC, T (&bNew)[2], const T (&bOld)[2], FlagRows& fl,
                  DynRow<T>& dc) {
    const int yA = y0 - yoff + k;
    if (PRIO_PHASE || (PRIO_HALF0_PHASE && half == 0)) __builtin_amdgcn_s_setprio(1);  // stages A and B first
    if (WALLS && (yA == 1 || yA == 2)) {
      // a branch taken once per sweep (the asm statement keeps the compiler
      // from turning it into selects on every row)
      __asm__ volatile("" ::: "memory");
      if (yA == 1) rm = rc;              // delta-rho: centre value
      else vm = mirrored(vc);            // velocity fields: negated
    }

    // ---------------- stage A: moments of row yA ----------------
    const bool rowA = (WALLS ? (yA >= 0 && yA < ny) : true) && (half == 0 || yA >= y0 - 2);
    // rows of M (Eq. A1) applied to the deviations q; formed in each half's
    // branch so that the two sources of q need not share registers
    auto moments = [&](const T (&q)[9], T phi) {
      const T s13 = q[1] + q[3], s24 = q[2] + q[4];  // (shared with p_xx)
      const T sa = s13 + s24;
      const T sd = (q[5] + q[6]) + (q[7] + q[8]);
      rA.dm0 = q[0] + (sa + sd);
      rA.jx = (q[1] - q[3]) + ((q[5] - q[6]) + (q[8] - q[7]));
      rA.jy = (q[2] - q[4]) + ((q[5] + q[6]) - (q[7] + q[8]));
      rA.me = T(-4) * q[0] - sa + T(2) * sd;
      rA.mep = T(4) * q[0] - T(2) * sa + sd;
      rA.mqx = T(-2) * (q[1] - q[3]) + ((q[5] - q[6]) + (q[8] - q[7]));
      rA.mqy = T(-2) * (q[2] - q[4]) + ((q[5] + q[6]) - (q[7] + q[8]));
      rA.mpxx = s13 - s24;
      rA.mpxy = (q[5] + q[7]) - (q[6] + q[8]);
      rA.phi = phi;
      const T rp = recip(phi);
      if constexpr (!MASK) rA.rphi = rp;  // (recomputed with solid nodes: registers)
      rA.drho = rA.dm0 * rp;
    };
    // half 0: the staged row yA has landed once at most one batch (row
    // yA + 1: one load per staged word row) is still in flight
    if (half == 0) wait_vm<NW>();
    // the flags shift by one row on every iteration, whether or not the row
    // of stage A exists (stages B and C still do)
    if (MASK && half == 0) {
      // the flags of row yA + 2, staged with row yA
      const unsigned fnew = __builtin_bit_cast(unsigned, float((sl ? st1 : st0)->v[NW - 1][t]));
      __asm__ volatile("" ::: "memory");
      fl.hi = ((fl.hi << 10) | (fl.lo >> 10)) & 0x3FFFFFFFu;
      fl.lo = ((fl.lo << 10) | fnew) & 0xFFFFFu;
    } else if (MASK) {
      // those of row yA, with the row in half 0's ring (in bounds for every
      // row of the sweep; rows that do not exist give values never used)
      const unsigned nb = flags_of(L.pop[pop_slot(PL_NB, jr(yA))][t]);
      fl.hi = ((fl.hi << 10) | nb) & 0x3FFFFFFFu;
    }
    // A moving phi: half 0 takes the second step's phi(t+1), phi(t+2) and
    // beta of row yA from its staged row here, and after the first barrier
    // puts those of row yA - 1 (kept from the last iteration) into the ring:
    // the ring row of yA - 1 then holds row yA - 5, half 1's row of this
    // iteration, which it read before that barrier.
    T dyn_phi1 = T(0), dyn_phi2 = T(0), dyn_beta2 = T(0);
    if (DYN && half == 0) {
      const auto* st = sl ? st1 : st0;
      dyn_phi1 = staged<T>(st, V_PHIN, t);
      dyn_phi2 = staged<T>(st, V_PHIN2, t);
      if (DRAG) dyn_beta2 = staged<T>(st, V_BETA2, t);
      __asm__ volatile("" ::: "memory");
    }
    // the force field of stage B's row, loaded into registers here so that
    // the loads land while stage A runs (they take no LDS)
    T fex = T(0), fey = T(0);
    if (FORCE) {
      const int yf = yA - 1;
      const unsigned ro = unsigned(WALLS ? min(max(yf, 0), ny - 1) : wrap_index(yf, ny)) * unsigned(pitch) * TB;
      // with a moving phi the second step (half 1) has a force field of its own
      fex = bload<T>((DYN && half) ? fx2r : fxr, xcT, ro);
      fey = bload<T>((DYN && half) ? fy2r : fyr, xcT, ro);
    }
    if (rowA) {
      if (half == 0) {
        S f[9];
        const auto* st = sl ? st1 : st0;
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = staged<S>(st, i, t);
        const T phi = staged<T>(st, 9, t);
        if (DRAG) rA.beta = staged<T>(st, 10, t);
        if (DYN) rA.dphi = dyn_phi1 - phi;  // d_t phi of the first step
        // keeps these reads here, next to the wait that orders them: merged
        // with half 1's read of phi they would wait for the row ahead too
        __asm__ volatile("" ::: "memory");
        T q[9];
        if (SHIFT) {
#pragma unroll
          for (int i = 0; i < 9; ++i) {
            // FP16: widened and scaled in one mixed-precision FMA (the product
            // of the exact widening rounds once, as a multiply would; only an
            // exact zero takes the sign of + 0)
            if constexpr (sizeof(S) == 2) q[i] = __builtin_fmaf(static_cast<float>(f[i]), ph.inv_scale, 0.0f);
            else q[i] = static_cast<T>(f[i]);
          }
        } else {
          q[0] = static_cast<T>(f[0]) - (phi * rho0 - ph.rest0_k);
#pragma unroll
          for (int i = 1; i < 5; ++i) q[i] = static_cast<T>(f[i]) - ph.rest_axis;
#pragma unroll
          for (int i = 5; i < 9; ++i) q[i] = static_cast<T>(f[i]) - ph.rest_diag;
        }
        moments(q, phi);
      } else {
        // pull from half 0's ring: f_i(x) = f+_i(x - e_i); at a wall the
        // image rows hold the bounced-back populations.  phi of the row came
        // with it.
        // One address per ring row (the lane's column in plane 0); the planes
        // and the column shifts are immediate offsets.  At lanes 0 and NT - 1
        // the shifted reads fall on the edge of a neighbouring ring row, still
        // inside the ring (no shifted plane is the ring's first or last); the
        // moments of those lanes are not valid for half 1 and never used.
        T q[9];
        const int j0 = jr(yA);
        const auto* r0 = &L.pop[0][0] + (j0 & 3) * NT + t;
        const auto* rm = &L.pop[0][0] + ((j0 - 1) & 3) * NT + t;
        const auto* rp = &L.pop[0][0] + ((j0 + 1) & 3) * NT + t;
        constexpr int P = 4 * NT;  // elements per plane of the ring
        const T phi = r0[9 * P];
        if (DRAG) rA.beta = r0[10 * P];
        if (DYN) rA.dphi = r0[PL_PHIN2 * P] - phi;  // d_t phi of the second step
        q[0] = r0[0];
        q[1] = r0[1 * P - 1];
        q[3] = r0[3 * P + 1];
        q[2] = rm[2 * P];
        q[5] = rm[5 * P - 1];
        q[6] = rm[6 * P + 1];
        q[4] = rp[4 * P];
        q[7] = rp[7 * P + 1];
        q[8] = rp[8 * P - 1];
        if constexpr (MASK) {
          // a solid source: the own node's opposite population of the ring row
          const unsigned nb = fl.hi & 0x3FFu;
          if (wave_any((nb & BOUNCE) != 0)) {
            q[1] = solid_bit(nb, 3) ? r0[3 * P] : q[1];
            q[3] = solid_bit(nb, 1) ? r0[1 * P] : q[3];
            q[2] = solid_bit(nb, 4) ? r0[4 * P] : q[2];
            q[4] = solid_bit(nb, 2) ? r0[2 * P] : q[4];
            q[5] = solid_bit(nb, 7) ? r0[7 * P] : q[5];
            q[7] = solid_bit(nb, 5) ? r0[5 * P] : q[7];
            q[6] = solid_bit(nb, 8) ? r0[8 * P] : q[6];
            q[8] = solid_bit(nb, 6) ? r0[6 * P] : q[8];
          }
        }
        moments(q, phi);
      }
      // solid nodes: zero, left out of the separable sums
      s_rho[t] = (MASK && solid_bit(fl.hi, 0)) ? T(0) : rA.drho;
    } else if (WALLS && yA == ny) {
      // above the upper wall: row ny - 1 itself
      s_rho[t] = (MASK && solid_bit(fl.hi, 10)) ? T(0) : rB.drho;
    }
    lds_barrier();

    // The staging slot of row yA has been read (the barrier above waited for
    // this wave's LDS reads): it takes row yA + 2.
    // With FP16 storage (the pipeline, not HBM, bounds it) the loads of the
    // rows below and above follow the second barrier: the phase between the
    // barriers is the short one.  (With 4-byte storage the later half loses
    // more to the shorter time in flight; with the force field its register
    // loads' wait would cover those loads too.)
    constexpr bool SPLIT = sizeof(S) == 2 && !MASK && !FORCE;
    if (half == 0) stage_row(yA + 2, sl, fl.lo & 0x3FFu, SPLIT ? 1 : 0);
    if (DYN && half == 0) {
      const int ja = jr(yA - 1);
      L.pop[pop_slot(9, ja)][t] = dc.phi1;
      L.pop[pop_slot(PL_PHIN2, ja)][t] = dc.phi2;
      if (DRAG) L.pop[pop_slot(10, ja)][t] = dc.beta2;
      dc.phi1 = dyn_phi1;
      dc.phi2 = dyn_phi2;
      dc.beta2 = dyn_beta2;
    }

    // ---------------- stage B: velocity of row yA - 1 ----------------
    // D and S of delta-rho on row yA, then grad rho on row yA - 1.  D and S
    // of rows that do not exist are never used.
    const int yb = yA - 1;
    const bool rowB = (WALLS ? (yb >= 0 && yb < ny) : true) && (yb >= y0 - 4 + 3 * half);
    {
      RhoDS<T> rn;
      {
        const T r0 = s_rho[t], rE = s_rho[tr], rW = s_rho[tl];
        rn.d = rE - rW;
        rn.s = (rE + rW) + T(4) * r0;
      }
      if (rowB) {
        T grx = T(4) * rc.d + (rm.d + rn.d);  // 12 d_x rho (Eq. 10)
        T gry = rn.s - rm.s;                  // 12 d_y rho
        if constexpr (MASK) {
          const unsigned nbB = (fl.hi >> 10) & 0x3FFu;
          if (wave_any((nbB & BOUNCE) != 0)) {  // solid neighbours: the centre value
            grx += T(solid_kx(nbB)) * rB.drho;
            gry += T(solid_ky(nbB)) * rB.drho;
          }
        }
        const T phi = rB.phi;
        const T kp = (kappa - (kappa_less_one ? T(1) : phi)) * T(1.0 / 36.0);  // Eq. (13), with the 1/12
        const T sg = ph.scale_by_phi ? phi : T(1);
        T Fx = kp * grx + sg * ph.gx;
        T Fy = kp * gry + sg * ph.gy;
        if (FORCE) {
          Fx += fex;
          Fy += fey;
        }
        const T m0 = phi * rho0 + rB.dm0;
        T ux, uy;
        if (DRAG) {
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
        if (MASK && solid_bit(fl.hi, 10)) {  // solid node: zero, left out of the sums
          a.ux = a.uy = a.mux = a.rux = T(0);
          b.muy = b.ruy = T(0);
        }
        lds_put(s_u4[t], a);
        lds_put(s_u2[t], b);
        bNew[0] = Fx;
        bNew[1] = Fy;
      } else if (WALLS && yb == ny) {  // above the upper wall: row ny - 1, negated
        U4<T> a = lds_get(s_u4[t]);
        U2<T> b = lds_get(s_u2[t]);
        a.ux = -a.ux; a.uy = -a.uy; a.mux = -a.mux; a.rux = -a.rux;
        b.muy = -b.muy; b.ruy = -b.ruy;
        lds_put(s_u4[t], a);
        lds_put(s_u2[t], b);
      }
      rm = rc;
      rc = rn;
    }
    lds_barrier();
    if (PRIO_PHASE || (PRIO_HALF0_PHASE && half == 0)) __builtin_amdgcn_s_setprio(0);  // stage C after them

    if (SPLIT && half == 0) stage_row(yA + 2, sl, 0u, 2);

    // ---------------- stage C: collide row yA - 2 ----------------
    const int yo = yA - 2;
    const bool rowC = (WALLS ? (yo >= 0 && yo < ny) : true) &&
                      (half == 0 ? (yo >= y0 - 3 && yo <= y1 + 2) : (yo >= y0 && yo < y1));
    if (WALLS && half == 0 && (yo == 1 || yo == ny) && olane) {
      // Image rows of the population ring for half 1's pull next to a wall
      // (half-way bounce-back: the population leaving x across the wall
      // returns to x in the opposite direction).  Written one iteration after
      // the wall row, into ring rows that nothing reads until half 1 pulls
      // the wall row.  Position t takes the value of the lane that the pull
      // at t - e_i stands for.
      const int js = jr(yo - 1);  // the wall row
      if (yo == 1) {  // row -1 from row 0
        const int jd = js - 1;
        const T v2 = L.pop[pop_slot(4, js)][t];
        const T v5 = L.pop[pop_slot(7, js)][tr];
        const T v6 = L.pop[pop_slot(8, js)][tl];
        L.pop[pop_slot(2, jd)][t] = v2;
        L.pop[pop_slot(5, jd)][t] = v5;
        L.pop[pop_slot(6, jd)][t] = v6;
      } else {        // row ny from row ny - 1
        const int jd = js + 1;
        const T v4 = L.pop[pop_slot(2, js)][t];
        const T v7 = L.pop[pop_slot(5, js)][tl];
        const T v8 = L.pop[pop_slot(6, js)][tr];
        L.pop[pop_slot(4, jd)][t] = v4;
        L.pop[pop_slot(7, jd)][t] = v7;
        L.pop[pop_slot(8, jd)][t] = v8;
      }
    }
    {
      // D and S of the velocity fields on row yb
      VelDS<T> vn;
      {
        const U4<T> a0 = lds_get(s_u4[t]), aE = lds_get(s_u4[tr]), aW = lds_get(s_u4[tl]);
        const U2<T> b0 = lds_get(s_u2[t]), bE = lds_get(s_u2[tr]), bW = lds_get(s_u2[tl]);
        vn.d_rux = aE.rux - aW.rux;
        vn.d_ux = aE.ux - aW.ux;
        vn.d_uy = aE.uy - aW.uy;
        vn.d_mux = aE.mux - aW.mux;
        vn.s_ruy = (bE.ruy + bW.ruy) + T(4) * b0.ruy;
        vn.s_uy = (aE.uy + aW.uy) + T(4) * a0.uy;
        vn.s_ux = (aE.ux + aW.ux) + T(4) * a0.ux;
        vn.s_muy = (bE.muy + bW.muy) + T(4) * b0.muy;
        vn.ux = a0.ux;
        vn.uy = a0.uy;
        if constexpr (EQ2) {
          vn.d_ruy = bE.ruy - bW.ruy;
          vn.d_muy = bE.muy - bW.muy;
          vn.s_rux = (aE.rux + aW.rux) + T(4) * a0.rux;
          vn.s_mux = (aE.mux + aW.mux) + T(4) * a0.mux;
        }
      }
      if (rowC && olane) {
        // the eight derivatives of Eq. (20), each 12 times its Eq. (10) value
        const T dx_rux = T(4) * vc.d_rux + (vm.d_rux + vn.d_rux);
        const T dx_ux = T(4) * vc.d_ux + (vm.d_ux + vn.d_ux);
        const T dx_uy = T(4) * vc.d_uy + (vm.d_uy + vn.d_uy);
        const T dx_mux = T(4) * vc.d_mux + (vm.d_mux + vn.d_mux);
        const T dy_ruy = vn.s_ruy - vm.s_ruy;
        const T dy_uy = vn.s_uy - vm.s_uy;
        const T dy_ux = vn.s_ux - vm.s_ux;
        const T dy_muy = vn.s_muy - vm.s_muy;

        const T phi = rC.phi;
        const T rho = rho0 + rC.drho;
        const T m0 = phi * rho0 + rC.dm0;
        const T X = kappa * (MASK ? recip(phi) : rC.rphi);
        const T kr = (kappa - (kappa_less_one ? T(1) : phi)) * rho;
        const T ux = vc.ux, uy = vc.uy, Fx = bOld[0], Fy = bOld[1];

        // penalty source (Eq. 20), static void fraction; the 1/12 of the
        // derivatives is folded into the coefficients
        T Ca, Cb, Cc;
        if constexpr (EQ2) {
          // Eq. (B3): twice the kappa and the phi rho u terms of Ca, two
          // thirds of those of Cb, and Cc with all three kinds of term
          const T dx_ruy = T(4) * vc.d_ruy + (vm.d_ruy + vn.d_ruy);
          const T dx_muy = T(4) * vc.d_muy + (vm.d_muy + vn.d_muy);
          const T dy_rux = vn.s_rux - vm.s_rux;
          const T dy_mux = vn.s_mux - vm.s_mux;
          Ca = T(-2) * ph.k12 * (dx_rux + dy_ruy) + (kr * T(1.0 / 6.0)) * (dx_ux + dy_uy) +
               (T(1.0 / 3.0) - X * T(1.0 / 6.0)) * (dx_mux + dy_muy);
          Cb = T(-2.0 / 3.0) * ph.k12 * (dx_rux - dy_ruy) + (kr * T(1.0 / 18.0)) * (dx_ux - dy_uy) +
               T(1.0 / 18.0) * (dx_mux - dy_muy);
          Cc = T(-1.0 / 3.0) * ph.k12 * (dx_ruy + dy_rux) + (kr * T(1.0 / 36.0)) * (dx_uy + dy_ux) +
               T(1.0 / 36.0) * (dx_muy + dy_mux);
        } else {
          Ca = -ph.k12 * (dx_rux + dy_ruy) + (kr * T(1.0 / 6.0)) * (dx_ux + dy_uy) +
               (T(0.25) - X * T(1.0 / 6.0)) * (dx_mux + dy_muy);
          Cb = -ph.k12 * (dx_rux - dy_ruy) + (kr * T(1.0 / 18.0)) * (dx_ux - dy_uy) +
               T(1.0 / 12.0) * (dx_mux - dy_muy);
          Cc = (kr * T(1.0 / 36.0)) * (dx_uy + dy_ux);
        }
        if (DYN) Ca -= T(2) * X * rho * rC.dphi;  // moving phi (Eq. 20)
        if constexpr (MASK) {
          const unsigned nbC = (fl.hi >> 20) & 0x3FFu;
          if (wave_any((nbC & BOUNCE) != 0)) {
            // Solid neighbours stand in with the centre's velocity-like
            // fields negated: each derivative gains -Kx (or -Ky) times the
            // centre's rho u, u or (phi rho) u, here gathered into the three
            // sums (rho u = rho (u), (phi rho) u = m0 (u))
            const T kx = T(solid_kx(nbC)), ky = T(solid_ky(nbC));
            const T sp = kx * ux + ky * uy, sm = kx * ux - ky * uy, sc = kx * uy + ky * ux;
            if constexpr (EQ2) {  // the same with the coefficients of Eq. (B3)
              Ca -= sp * ((kr * T(1.0 / 6.0) - T(2) * ph.k12 * rho) + (T(1.0 / 3.0) - X * T(1.0 / 6.0)) * m0);
              Cb -= sm * ((kr * T(1.0 / 18.0) - T(2.0 / 3.0) * ph.k12 * rho) + T(1.0 / 18.0) * m0);
              Cc -= sc * ((kr * T(1.0 / 36.0) - T(1.0 / 3.0) * ph.k12 * rho) + T(1.0 / 36.0) * m0);
            } else {
              Ca -= sp * ((kr * T(1.0 / 6.0) - ph.k12 * rho) + (T(0.25) - X * T(1.0 / 6.0)) * m0);
              Cb -= sm * ((kr * T(1.0 / 18.0) - ph.k12 * rho) + T(1.0 / 12.0) * m0);
              Cc -= sc * (kr * T(1.0 / 36.0));
            }
          }
        }

        // equilibria (Eq. 18) minus those of the rest state
        const T drho = rC.drho;
        const T uu = ux * ux + uy * uy;
        const T eq_e = (ph.k2 - T(4) * phi) * drho + T(3) * m0 * uu;
        const T eq_ep = (T(4) * phi - ph.k3) * drho - T(3) * m0 * uu;
        const T qfac = EQ2 ? -m0 : (kappa - T(2) * phi) * rho;  // phi rho (X - 2), or -phi rho (B2)
        const T eq_qx = qfac * ux, eq_qy = qfac * uy;
        const T eq_pxx = m0 * (ux * ux - uy * uy);
        const T eq_pxy = m0 * (ux * uy);

        // force moments (Eq. 19)
        const T uF = ux * Fx + uy * Fy;
        const T S1 = T(6) * uF;
        const T S7 = T(2) * (ux * Fx - uy * Fy);
        const T S8 = ux * Fy + uy * Fx;

        // relaxation (Eq. 16); conserved moments: m0+ = m0, j+ = j + F
        const T he = ph.he, hep = ph.hep, hq = ph.hq, hn = ph.hn;
        const T pe = rC.me - ph.s_e * (rC.me - eq_e) + he * (S1 + Ca);
        const T pep = rC.mep - ph.s_eps * (rC.mep - eq_ep) - hep * S1;
        const T pqx = rC.mqx - ph.s_q * (rC.mqx - eq_qx) - hq * Fx;
        const T pqy = rC.mqy - ph.s_q * (rC.mqy - eq_qy) - hq * Fy;
        const T ppxx = rC.mpxx - ph.s_nu * (rC.mpxx - eq_pxx) + hn * (S7 + Cb);
        const T ppxy = rC.mpxy - ph.s_nu * (rC.mpxy - eq_pxy) + hn * (S8 + Cc);
        const T pm0 = rC.dm0;
        const T pjx = rC.jx + Fx;
        const T pjy = rC.jy + Fy;

        // back-transform f+ = M^-1 m+ (Eq. A1).  Half 1 with shifted storage
        // takes the coefficients times the storage scale (a power of two, so
        // the products are the scaled values exactly, as a multiply at the
        // store would give them).
        const bool scaled = SHIFT && half != 0;
        const T c36 = scaled ? ph.bt36 : T(1.0 / 36.0), c6 = scaled ? ph.bt6 : T(1.0 / 6.0);
        const T c12 = scaled ? ph.bt12 : T(1.0 / 12.0), c4 = scaled ? ph.bt4 : T(0.25);
        const T c9 = scaled ? ph.bt9 : T(1.0 / 9.0);
        const T a = (T(4) * pm0 - pe - T(2) * pep) * c36;
        const T b = (T(4) * pm0 + T(2) * pe + pep) * c36;
        const T X1 = (pjx - pqx) * c6, Y1 = (pjy - pqy) * c6;
        const T X2 = (T(2) * pjx + pqx) * c12, Y2 = (T(2) * pjy + pqy) * c12;
        const T Pd = ppxx * c4, Qd = ppxy * c4;
        T o9[9];
        o9[0] = (pm0 - pe + pep) * c9;
        // the rows of M^-1 by their shared pairs: six additions fewer than
        // summing each row's terms in turn
        const T aP = a + Pd, aM = a - Pd, bP = b + Qd, bM = b - Qd;
        const T sXY = X2 + Y2, dXY = X2 - Y2;
        o9[1] = aP + X1;
        o9[2] = aM + Y1;
        o9[3] = aP - X1;
        o9[4] = aM - Y1;
        o9[5] = bP + sXY;
        o9[6] = bM - dXY;
        o9[7] = bP - sXY;
        o9[8] = bM + dXY;
        if (MASK && solid_bit(fl.hi, 20)) {  // solid node: keep the rest state
#pragma unroll
          for (int i = 0; i < 9; ++i) o9[i] = T(0);
        }
        // a moving phi: the ring and shifted storage hold deviations from the
        // rest state of the void fraction the next pull runs at, whose rest_0
        // is rho0 d_t phi higher (times the storage scale for half 1's stores)
        if (DYN && (half == 0 || SHIFT)) o9[0] -= (scaled ? ph.scale : T(1)) * (rho0 * rC.dphi);

        if (half == 0) {  // into the ring for the second step
          const int jo = jr(yo);
#pragma unroll
          for (int i = 0; i < 9; ++i) L.pop[pop_slot(i, jo)][t] = o9[i];
          if (!DYN) {  // (with a moving phi, written with the row's staging)
            L.pop[pop_slot(9, jo)][t] = phi;
            if (DRAG) L.pop[pop_slot(10, jo)][t] = rC.beta;
          }
          if (MASK) L.pop[pop_slot(PL_NB, jo)][t] = flags_as<T>((fl.hi >> 20) & 0x3FFu);
        } else if (SHIFT) {  // already scaled
#pragma unroll
          for (int i = 0; i < 9; ++i) bstore(static_cast<S>(o9[i]), dstr, xcb, poff(i, yo));
        } else {
          bstore(static_cast<S>(o9[0] + (phi * rho0 - ph.rest0_k)), dstr, xcb, poff(0, yo));
#pragma unroll
          for (int i = 1; i < 5; ++i) bstore(static_cast<S>(o9[i] + ph.rest_axis), dstr, xcb, poff(i, yo));
#pragma unroll
          for (int i = 5; i < 9; ++i) bstore(static_cast<S>(o9[i] + ph.rest_diag), dstr, xcb, poff(i, yo));
        }
      }
      vm = vc;
      vc = vn;
    }
    // The end of the iteration: no barrier.  Half 0's collision row yo is
    // pulled by half 1 LAG - 3 = two iterations later, behind the next
    // iteration's barriers, and its ring slot is that of row yo - 4, which
    // half 1 read before this iteration's first barrier.  The next
    // iteration's stage A writes the delta-rho row after every wave has
    // passed this iteration's second barrier (its stage B reads done), and
    // its stage B writes the velocity row after its first barrier (this
    // stage C's reads done).
  };

  // Software pipeline: half 0 stages rows two ahead (see stage_row); the
  // loop is unrolled by six (a multiple of the three-row period of the
  // states and of the two staging slots) so nothing is copied.  With solid
  // nodes the flags of the first two rows are loaded here.
  RowState<T> R0{}, R1{}, R2{};
  T b0[2] = {0, 0}, b1[2] = {0, 0};
  FlagRows fl{0u, 0u};
  DynRow<T> dc{T(0), T(0), T(0)};
  if (half == 0) {
    unsigned fa = 0, fb = 0;
    if (MASK) {
      fa = bload_u16(nbrr, unsigned(c) * 2u, flag_row(y0 - 7));
      fb = bload_u16(nbrr, unsigned(c) * 2u, flag_row(y0 - 6));
      fl.lo = fb | (fa << 10);
    }
    stage_row(y0 - 5, 0, fa);
    stage_row(y0 - 4, 1, fb);
  }
  for (int k = 0; k < nit; k += 6) {
    body(k + 0, 0, R0, R2, R1, b0, b1, fl, dc);
    if (k + 1 >= nit) break;
    body(k + 1, 1, R1, R0, R2, b1, b0, fl, dc);
    if (k + 2 >= nit) break;
    body(k + 2, 0, R2, R1, R0, b0, b1, fl, dc);
    if (k + 3 >= nit) break;
    body(k + 3, 1, R0, R2, R1, b1, b0, fl, dc);
    if (k + 4 >= nit) break;
    body(k + 4, 0, R1, R0, R2, b0, b1, fl, dc);
    if (k + 5 >= nit) break;
    body(k + 5, 1, R2, R1, R0, b1, b0, fl, dc);
  }
  // no load into LDS may outlive the workgroup
  wait_vm<0>();
}

// Two time steps per launch: workgroup b takes tile xcd_tile(b) (strip
// tile % strips, row block tile / strips); 2 NT lanes (two halves of NT),
// four waves per SIMD.
template <typename S, typename T, bool SHIFT, bool WALLS, int FEAT, int NT>
__global__ void __launch_bounds__(2 * NT) __attribute__((amdgpu_waves_per_eu(step2_waves<T, FEAT>())))
vanse_step2_kernel(StepGeom g, StepPhys<T> ph) {
  __shared__ Step2Lds<T, NT, step2_planes<FEAT>()> lds;
  __shared__ Step2Stage<NT, step2_words<S, FEAT>()> stage0, stage1;
  const int tile = xcd_tile(int(blockIdx.x), int(gridDim.x));
  step2_tile<S, T, SHIFT, WALLS, FEAT, NT>(g, ph, tile % g.strips, tile / g.strips,
                                           lds_handle(&lds), lds_handle(&stage0),
                                           lds_handle(&stage1));
}

// Many lattices, two time steps per launch: workgroup b takes the tile that
// entry xcd_tile(b) of the tile map names (lattice, and strip and row block
// as in the one-lattice kernel); each member's two buffers alternate with
// the launch parity as in the one-step batch.
template <typename S, typename T, bool SHIFT, bool WALLS, int FEAT, int NT>
__global__ void __launch_bounds__(2 * NT) __attribute__((amdgpu_waves_per_eu(step2_waves<T, FEAT>())))
vanse_batch_step2_kernel(const BatchEntry<T>* __restrict__ entries,
                         const int2* __restrict__ tile_map, int launch) {
  __shared__ Step2Lds<T, NT, step2_planes<FEAT>()> lds;
  __shared__ Step2Stage<NT, step2_words<S, FEAT>()> stage0, stage1;
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
  // a private copy, as the one-lattice kernel's argument: read through the
  // table the parameters could alias the stores as far as the compiler knows
  const StepPhys<T> ph = e.ph;
  step2_tile<S, T, SHIFT, WALLS, FEAT, NT>(g, ph, local % g.strips, local / g.strips,
                                           lds_handle(&lds), lds_handle(&stage0),
                                           lds_handle(&stage1));
}

}  // namespace vanse_dev
