/*
 * vanse_oracle.c -- plain FP64 CPU reference for one time step of the
 * consistent multiple-relaxation-time lattice Boltzmann method for the
 * volume-averaged Navier-Stokes equations (MRTLB-VANSE) on a D2Q9 lattice,
 * after Liu, Zhang, Min & Wu, arXiv:2409.02964.
 *
 * TEST INFRASTRUCTURE.  This file is the oracle that the GPU path is checked
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header, table or helper with the
 * GPU library, and the product never calls it.
 *
 * Style: slow and literal on purpose.  Whole-field passes in the order the
 * paper states the scheme (Sec. 2.3), the 9x9 matrices of Eq. (A1) applied as
 * plain matrix-vector products, push streaming into a fresh array, no fusion,
 * no blocking.  Build with -O3 -ffp-contract=off and without -ffast-math,
 * so there is no FMA contraction and no reassociation.  The per-node loops
 * may run on several OpenMP threads; no loop reduces across nodes, so the
 * results do not depend on the thread count.
 *
 * Layout: every field is row-major [ny][nx], index y*nx + x.  Populations
 * are nine such planes, plane i at f + i*nx*ny.  The state held between
 * steps is the post-streaming (pre-collision) population f_i(x, t).
 *
 * Readings of the paper taken here (each one is listed in the design notes):
 *  - the paper's tau_* are relaxation RATES (Sec. 2.2: tau^-1 = nu/cs^2+1/2
 *    for SRT; Eq. (A11) for MRT); they are called s_* here;
 *  - gradients of Eq. (13) and Eq. (20) use fields of the same time level,
 *    computed from the current populations, neighbour velocities included;
 *  - derivatives of products (e.g. d_x(rho u_x)) apply Eq. (10) to the
 *    node-wise product field; phi*rho*u is formed as (sum_i f_i) * u, since
 *    Eq. (7) defines phi*rho as the zeroth moment;
 *  - d_t phi is the forward difference phi(t+1) - phi(t) (Sec. 2.3, below
 *    Eq. (20)); it is zero when no next field is given;
 *  - Eq. (10) next to a domain wall uses the mirror image across the wall
 *    (scalars copied, velocity-like fields negated, i.e. zero at the
 *    half-way wall); next to a solid node of the mask it uses the centre
 *    node's own value (velocity-like fields negated);
 *  - walls are half-way bounce-back (Sec. 3.1) on the domain faces, so every
 *    stored row/column is fluid unless the mask says otherwise;
 *  - the body force is F^B = phi*G + F_ext when scale_by_phi is set (the
 *    paper's F^B = phi(G - ...) form, Sec. 3.1 and Eq. (23)), else G + F_ext.
 *  - Eq. (16) is taken with a minus sign on the relaxation term (Eq. (A2)
 *    prints a plus, at odds with Eq. (16) and Eq. (A3)).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- lattice constants, Eq. (5) ------------------------------------------ */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WT[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
#define CS2 (1.0 / 3.0) /* lattice sound speed squared, c = 1 */

/* ---- transformation matrix and its inverse, Eq. (A1) ---------------------- */
/* moment order (Eq. 17): (phi*rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy) */
static const double MM[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};
/* M^-1 = (1/36) * MINV36, as printed in Eq. (A1) */
static const double MINV36[9][9] = {
    {4, -4, 4, 0, 0, 0, 0, 0, 0},   {4, -1, -2, 6, -6, 0, 0, 9, 0},
    {4, -1, -2, 0, 0, 6, -6, -9, 0}, {4, -1, -2, -6, 6, 0, 0, 9, 0},
    {4, -1, -2, 0, 0, -6, 6, -9, 0}, {4, 2, 1, 6, 3, 6, 3, 0, 9},
    {4, 2, 1, -6, -3, 6, 3, 0, -9}, {4, 2, 1, -6, -3, -6, -3, 0, 9},
    {4, 2, 1, 6, 3, -6, -3, 0, -9}};

typedef struct {
  int nx, ny;
  int bc_x, bc_y;  /* 0 periodic, 1 half-way bounce-back walls on both faces */
  double kappa;    /* provisional equation-of-state constant, Eq. (13) */
  double s_c, s_e, s_eps, s_q, s_nu; /* diagonal of Gamma, Eq. (16) */
  double gx, gy;   /* uniform external acceleration G */
  int scale_by_phi;/* 1: F^B = phi*G (+F_ext); 0: F^B = G (+F_ext) */
  int use_penalty; /* 1: penalty source C of Eq. (20); 0: ablation (tests) */
  /* Linear drag towards a solid velocity u_s: F^B gains -phi*beta*(u - u_s)
   * (the Darcy term of Eq. (21), beta = phi*nu/k0, and the particle drag of
   * Eq. (23), beta = phi*(1 - phi)).  NULL: no drag. */
  const double *beta;
  double usx, usy;
  /* Model B (set I), Sec. 2.3 below Eq. (20): F^p = (kappa - 1) cs^2 grad rho
   * and "kappa - phi" -> "kappa - 1" in the source term. */
  int model_b;
  /* 1: the second-order equilibrium of Appendix B (B1, moments B2) with the
   * source term B3 in place of Eq. (14)/(18)/(20). */
  int eq2;
  /* Tangential (x) velocities of the walls on the faces y = -1/2 (lo) and
   * y = ny - 1/2 (hi), and the density rho_w of the moving-wall bounce-back:
   * a population f+_i crossing a wall returns as f_opp(i) = f+_i - (f^eq_i -
   * f^eq_opp(i)) at (phi(x), rho_w, u_w), and the Eq. (10) stand-in across the
   * wall carries 2 u_w - u (Sec. 3.1, Couette flow of Eq. 22). */
  double uw_lo, uw_hi, rho_w;
  /* Velocity boundary of Couette flow by non-equilibrium extrapolation
   * (Sec. 3.1, the paper's ref. [47]): nee_lo / nee_hi make the first / last
   * row a row of boundary nodes lying on the wall, moving with x velocity
   * un_lo / un_hi.  Needs bc_y = 1 and at least three rows.  Such a node is
   * not evolved by the scheme: after every collision its post-collision
   * populations are the equilibrium at (phi(x_b), rho(x_f), u_w) plus the
   * post-collision non-equilibrium part of its fluid neighbour x_f across the
   * row (f+ - f^eq at (phi(x_f), rho(x_f), u(x_f))), with the density
   * extrapolated as rho(x_b) = rho(x_f).  The Eq. (10) stencils of x_f see
   * rho(x_b) = rho(x_f) and u(x_b) = u_w there. */
  int nee_lo, nee_hi;
  double un_lo, un_hi;
} vo_params;

/* Boundary-row kind of row y: 1 lower, 2 upper velocity row, 0 otherwise. */
static int nee_row(const vo_params *P, int y) {
  if (P->bc_y == 0) return 0;
  if (P->nee_lo && y == 0) return 1;
  if (P->nee_hi && y == P->ny - 1) return 2;
  return 0;
}

/* ---- threads ------------------------------------------------------------- */
void vo_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int vo_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ---- small exported helpers (used by the identity tests) ----------------- */

void vo_tables(double *M, double *Minv36, int *ex, int *ey, double *w,
               int *opp) {
  for (int i = 0; i < 9; ++i) {
    for (int j = 0; j < 9; ++j) {
      M[i * 9 + j] = MM[i][j];
      Minv36[i * 9 + j] = MINV36[i][j];
    }
    ex[i] = EX[i];
    ey[i] = EY[i];
    w[i] = WT[i];
    opp[i] = OPP[i];
  }
}

/* Adjusted density equilibrium with the provisional equation of state,
 * third-order Hermite form, Eq. (14).  X = kappa/phi. */
void vo_feq(double phi, double rho, double ux, double uy, double kappa,
            double *feq) {
  const double X = kappa / phi;
  const double uu = ux * ux + uy * uy;
  double sum_w_nonzero = 0.0;
  for (int i = 1; i < 9; ++i) sum_w_nonzero += WT[i];
  feq[0] = phi * rho - sum_w_nonzero * kappa * rho -
           WT[0] * phi * rho * uu / (2.0 * CS2);
  for (int i = 1; i < 9; ++i) {
    const double eu = EX[i] * ux + EY[i] * uy;
    const double ee = (double)(EX[i] * EX[i] + EY[i] * EY[i]);
    const double third = 1.0 + 0.5 * (X - 1.0) * (ee / CS2 - 4.0);
    feq[i] = WT[i] * (kappa * rho +
                      phi * rho *
                          (eu / CS2 * third + eu * eu / (2.0 * CS2 * CS2) -
                           uu / (2.0 * CS2)));
  }
}

/* Equilibrium moments, Eq. (18). */
void vo_meq(double phi, double rho, double ux, double uy, double kappa,
            double *meq) {
  const double X = kappa / phi;
  const double pr = phi * rho;
  const double uu = ux * ux + uy * uy;
  meq[0] = pr * 1.0;
  meq[1] = pr * (-4.0 + 3.0 * uu + 2.0 * X);
  meq[2] = pr * (4.0 - 3.0 * uu - 3.0 * X);
  meq[3] = pr * ux;
  meq[4] = pr * (X - 2.0) * ux;
  meq[5] = pr * uy;
  meq[6] = pr * (X - 2.0) * uy;
  meq[7] = pr * (ux * ux - uy * uy);
  meq[8] = pr * (ux * uy);
}

/* Equilibrium moments of the second-order equilibrium, Eq. (B2): those of
 * Eq. (18) except the energy-flux rows, which are -phi rho u. */
void vo_meq2(double phi, double rho, double ux, double uy, double kappa,
             double *meq) {
  const double X = kappa / phi;
  const double pr = phi * rho;
  const double uu = ux * ux + uy * uy;
  meq[0] = pr;
  meq[1] = pr * (-4.0 + 3.0 * uu + 2.0 * X);
  meq[2] = pr * (4.0 - 3.0 * uu - 3.0 * X);
  meq[3] = pr * ux;
  meq[4] = -pr * ux;
  meq[5] = pr * uy;
  meq[6] = -pr * uy;
  meq[7] = pr * (ux * ux - uy * uy);
  meq[8] = pr * (ux * uy);
}

/* Force moments S = M F of Guo's forcing, Eq. (19). */
void vo_force_moments(double ux, double uy, double Fx, double Fy, double *S) {
  const double uF = ux * Fx + uy * Fy;
  S[0] = 0.0;
  S[1] = 6.0 * uF;
  S[2] = -6.0 * uF;
  S[3] = Fx;
  S[4] = -Fx;
  S[5] = Fy;
  S[6] = -Fy;
  S[7] = 2.0 * (ux * Fx - uy * Fy);
  S[8] = ux * Fy + uy * Fx;
}

/* Penalty source components (C_a, C_b, C_c) of Eq. (20). d[] holds
 * d_x(rho u_x), d_y(rho u_y), d_x u_x, d_y u_y, d_x u_y, d_y u_x,
 * d_x(phi rho u_x), d_y(phi rho u_y) at the node. */
/* kmp stands for the factor "kappa - phi" of Eq. (20): kappa - phi for the
 * consistent VANSE, kappa - 1 for model B. */
static void penalty20(double phi, double rho, double kappa, double kmp,
                      double dt_phi, const double *d, double *Cabc) {
  const double X = kappa / phi;
  const double drux_x = d[0], druy_y = d[1], dux_x = d[2], duy_y = d[3];
  const double duy_x = d[4], dux_y = d[5], dmux_x = d[6], dmuy_y = d[7];
  Cabc[0] = -kappa * (drux_x + druy_y) +
            2.0 * kmp * rho * (dux_x + duy_y) +
            (3.0 - 2.0 * X) * (dmux_x + dmuy_y) - 2.0 * X * rho * dt_phi;
  Cabc[1] = -kappa * (drux_x - druy_y) +
            2.0 / 3.0 * kmp * rho * (dux_x - duy_y) +
            (dmux_x - dmuy_y);
  Cabc[2] = 1.0 / 3.0 * kmp * rho * (duy_x + dux_y);
}

void vo_penalty(double phi, double rho, double kappa, double dt_phi,
                const double *d, double *Cabc) {
  penalty20(phi, rho, kappa, kappa - phi, dt_phi, d, Cabc);
}

/* Penalty source of Eq. (B3) for the second-order equilibrium.  d[] holds
 * the eight derivatives of Eq. (20) followed by d_x(rho u_y), d_y(rho u_x),
 * d_x(phi rho u_y), d_y(phi rho u_x). */
void vo_penalty_b3(double phi, double rho, double kappa, double kmp,
                   double dt_phi, const double *d, double *Cabc) {
  const double X = kappa / phi;
  const double drux_x = d[0], druy_y = d[1], dux_x = d[2], duy_y = d[3];
  const double duy_x = d[4], dux_y = d[5], dmux_x = d[6], dmuy_y = d[7];
  const double druy_x = d[8], drux_y = d[9], dmuy_x = d[10], dmux_y = d[11];
  Cabc[0] = -2.0 * kappa * (drux_x + druy_y) + 2.0 * kmp * rho * (dux_x + duy_y) +
            (4.0 - 2.0 * X) * (dmux_x + dmuy_y) - 2.0 * X * rho * dt_phi;
  Cabc[1] = -2.0 / 3.0 * kappa * (drux_x - druy_y) +
            2.0 / 3.0 * kmp * rho * (dux_x - duy_y) +
            2.0 / 3.0 * (dmux_x - dmuy_y);
  Cabc[2] = -kappa / 3.0 * (druy_x + drux_y) + 1.0 / 3.0 * kmp * rho * (duy_x + dux_y) +
            1.0 / 3.0 * (dmuy_x + dmux_y);
}

/* ---- neighbour lookup with the boundary/ghost rules ------------------------
 * Resolve the neighbour (x+dx, y+dy) of fluid node (x, y).  Returns the index
 * of the node whose value stands in for it, and sets *sign to -1 when the
 * stand-in is a reflection (velocity-like fields change sign there). */
static int is_solid(const unsigned char *mask, int idx) {
  return mask != NULL && mask[idx] != 0;
}

static int neighbour(const vo_params *P, const unsigned char *mask, int x,
                     int y, int dx, int dy, int *sign, int *wall) {
  int xn = x + dx, yn = y + dy;
  int reflected = 0;
  *wall = 0;
  if (xn < 0 || xn >= P->nx) {
    if (P->bc_x == 0) {
      xn = (xn + P->nx) % P->nx;
    } else {
      xn = (xn < 0) ? -1 - xn : 2 * P->nx - 1 - xn; /* image across the face */
      reflected = 1;
    }
  }
  if (yn < 0 || yn >= P->ny) {
    if (P->bc_y == 0) {
      yn = (yn + P->ny) % P->ny;
    } else {
      *wall = (yn < 0) ? 1 : 2;
      yn = (yn < 0) ? -1 - yn : 2 * P->ny - 1 - yn;
      reflected = 1;
    }
  }
  int idx = yn * P->nx + xn;
  if (is_solid(mask, idx)) { /* solid neighbour (at rest): centre value */
    idx = y * P->nx + x;
    reflected = 1;
    *wall = 0;
  }
  *sign = reflected ? -1 : 1;
  return idx;
}

/* Neighbour table: for every node c and direction i, the index standing in
 * for x+e_i and the sign for velocity-like fields (built once per step). */
typedef struct {
  int *idx;         /* [9][N] */
  signed char *sgn; /* [9][N] */
  signed char *wl;  /* [9][N]: 1 / 2 when the stand-in is across the lo / hi y-wall */
} vo_nbr;

static int nbr_build(const vo_params *P, const unsigned char *mask, vo_nbr *T) {
  const int N = P->nx * P->ny;
  T->idx = malloc((size_t)9 * N * sizeof(int));
  T->sgn = malloc((size_t)9 * N);
  T->wl = malloc((size_t)9 * N);
  if (!T->idx || !T->sgn || !T->wl) return -1;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < P->ny; ++y)
    for (int x = 0; x < P->nx; ++x)
      for (int i = 0; i < 9; ++i) {
        int sign, wall;
        const int c = y * P->nx + x;
        T->idx[(size_t)i * N + c] = neighbour(P, mask, x, y, EX[i], EY[i], &sign, &wall);
        T->sgn[(size_t)i * N + c] = (signed char)sign;
        T->wl[(size_t)i * N + c] = (signed char)wall;
      }
  return 0;
}

static void nbr_free(vo_nbr *T) {
  free(T->idx);
  free(T->sgn);
  free(T->wl);
}

/* Isotropic gradient, Eq. (10): d_a psi = 1/(cs^2 dt) sum_i w_i psi(x+e_i) e_ia.
 * odd = 1 for velocity-like fields (negated at reflected stand-ins).  xcomp
 * = 1 for the x component of a velocity-like field s u: across a moving wall
 * its stand-in is s (2 u_w - u), i.e. gains 2 u_w s, with s = 1 (scal NULL)
 * or scal at the image node. */
static void gradient_wall(const vo_params *P, const unsigned char *mask,
                          const vo_nbr *T, const double *psi, int odd, int xcomp,
                          const double *scal, double *gx, double *gy) {
  const int N = P->nx * P->ny;
#pragma omp parallel for schedule(static)
  for (int c = 0; c < N; ++c) {
    if (is_solid(mask, c)) {
      gx[c] = 0.0;
      gy[c] = 0.0;
      continue;
    }
    double sx = 0.0, sy = 0.0;
    for (int i = 0; i < 9; ++i) {
      const int n = T->idx[(size_t)i * N + c];
      double v = (odd && T->sgn[(size_t)i * N + c] < 0) ? -psi[n] : psi[n];
      const int wl = T->wl[(size_t)i * N + c];
      if (odd && xcomp && wl) {
        const double uw = (wl == 1) ? P->uw_lo : P->uw_hi;
        v += 2.0 * uw * (scal ? scal[n] : 1.0);
      }
      sx += WT[i] * v * EX[i];
      sy += WT[i] * v * EY[i];
    }
    gx[c] = sx / CS2;
    gy[c] = sy / CS2;
  }
}

static void gradient_tab(const vo_params *P, const unsigned char *mask,
                         const vo_nbr *T, const double *psi, int odd,
                         double *gx, double *gy) {
  gradient_wall(P, mask, T, psi, odd, 0, NULL, gx, gy);
}

void vo_gradient(const vo_params *P, const unsigned char *mask,
                 const double *psi, int odd, double *gx, double *gy) {
  vo_nbr T;
  if (nbr_build(P, mask, &T) == 0) gradient_tab(P, mask, &T, psi, odd, gx, gy);
  nbr_free(&T);
}

/* Work arrays of one step, allocated once per run. */
typedef struct {
  double *m0, *rho, *ux, *uy, *Fx, *Fy, *rux, *ruy, *mux, *muy, *d, *tmp;
  double *jx, *jy, *grx, *gry;
  double *fp; /* [9][N] post-collision populations of one step */
} vo_work;

static void work_free(vo_work *W) {
  free(W->m0); free(W->rho); free(W->ux); free(W->uy); free(W->Fx); free(W->Fy);
  free(W->rux); free(W->ruy); free(W->mux); free(W->muy); free(W->d); free(W->tmp);
  free(W->jx); free(W->jy); free(W->grx); free(W->gry); free(W->fp);
}

static int work_alloc(int N, vo_work *W) {
  const size_t b = (size_t)N * sizeof(double);
  W->m0 = malloc(b); W->rho = malloc(b); W->ux = malloc(b); W->uy = malloc(b);
  W->Fx = malloc(b); W->Fy = malloc(b); W->rux = malloc(b); W->ruy = malloc(b);
  W->mux = malloc(b); W->muy = malloc(b); W->d = malloc(12 * b); W->tmp = malloc(b);
  W->jx = malloc(b); W->jy = malloc(b); W->grx = malloc(b); W->gry = malloc(b);
  W->fp = malloc(9 * b);
  if (!W->m0 || !W->rho || !W->ux || !W->uy || !W->Fx || !W->Fy || !W->rux ||
      !W->ruy || !W->mux || !W->muy || !W->d || !W->tmp || !W->jx || !W->jy ||
      !W->grx || !W->gry || !W->fp) {
    work_free(W);
    return -1;
  }
  return 0;
}

/* ---- macroscopic fields, Eq. (7) with the force of Eq. (13) ---------------
 * rho = sum f / phi; grad rho by Eq. (10); F = (kappa - phi) cs^2 grad rho +
 * F^B; u = (sum e f + F/2) / sum f; p = rho cs^2.  Any output may be NULL. */
static void macroscopic_tab(const vo_params *P, const vo_nbr *T, vo_work *W,
                            const double *phi, const unsigned char *mask,
                            const double *fext_x, const double *fext_y,
                            const double *f, double *m0_out, double *rho_out,
                            double *ux_out, double *uy_out, double *Fx_out,
                            double *Fy_out, double *p_out) {
  const int N = P->nx * P->ny;
  /* the m0 and rho arrays double as outputs when the caller provides them */
  double *m0 = m0_out ? m0_out : W->tmp, *rho = rho_out ? rho_out : W->rho;
  double *jx = W->jx, *jy = W->jy, *grx = W->grx, *gry = W->gry;
#pragma omp parallel for schedule(static)
  for (int c = 0; c < N; ++c) {
    m0[c] = rho[c] = jx[c] = jy[c] = 0.0;
    if (is_solid(mask, c)) continue;
    double s = 0.0, sx = 0.0, sy = 0.0;
    for (int i = 0; i < 9; ++i) {
      const double fi = f[(size_t)i * N + c];
      s += fi;
      sx += EX[i] * fi;
      sy += EY[i] * fi;
    }
    m0[c] = s;
    jx[c] = sx;
    jy[c] = sy;
    rho[c] = s / phi[c];
  }
  /* velocity boundary rows: the density of the fluid neighbour across the
   * row, and phi*rho formed from it */
  if (P->nee_lo || P->nee_hi) {
    for (int y = 0; y < P->ny; ++y) {
      const int kind = nee_row(P, y);
      if (!kind) continue;
      const int yf = (kind == 1) ? 1 : P->ny - 2;
      for (int x = 0; x < P->nx; ++x) {
        const int c = y * P->nx + x;
        rho[c] = rho[yf * P->nx + x];
        m0[c] = phi[c] * rho[c];
      }
    }
  }
  gradient_tab(P, mask, T, rho, 0, grx, gry);
#pragma omp parallel for schedule(static)
  for (int c = 0; c < N; ++c) {
    double ux = 0.0, uy = 0.0, Fx = 0.0, Fy = 0.0;
    const int kind = nee_row(P, c / P->nx);
    if (kind) {
      ux = (kind == 1) ? P->un_lo : P->un_hi; /* the wall velocity; F unused */
    } else if (!is_solid(mask, c)) {
      /* Eq. (13); model B: F^p = (kappa - 1) cs^2 grad rho */
      const double kf = P->model_b ? 1.0 : phi[c];
      const double Fpx = (P->kappa - kf) * CS2 * grx[c];
      const double Fpy = (P->kappa - kf) * CS2 * gry[c];
      const double sc = P->scale_by_phi ? phi[c] : 1.0;
      double FBx = sc * P->gx, FBy = sc * P->gy;
      if (fext_x) FBx += fext_x[c];
      if (fext_y) FBy += fext_y[c];
      if (P->beta) {
        /* F depends on u through the drag: u = (j + F/2)/m0 with
         * F = F^p + F^B - phi beta (u - u_s), solved for u in closed form */
        const double d = phi[c] * P->beta[c];
        ux = (jx[c] + 0.5 * (Fpx + FBx + d * P->usx)) / (m0[c] + 0.5 * d);
        uy = (jy[c] + 0.5 * (Fpy + FBy + d * P->usy)) / (m0[c] + 0.5 * d);
        Fx = Fpx + FBx - d * (ux - P->usx);
        Fy = Fpy + FBy - d * (uy - P->usy);
      } else {
        Fx = Fpx + FBx;
        Fy = Fpy + FBy;
        ux = (jx[c] + 0.5 * Fx) / m0[c];
        uy = (jy[c] + 0.5 * Fy) / m0[c];
      }
    }
    if (m0_out) m0_out[c] = m0[c];
    if (rho_out) rho_out[c] = rho[c];
    if (ux_out) ux_out[c] = ux;
    if (uy_out) uy_out[c] = uy;
    if (Fx_out) Fx_out[c] = Fx;
    if (Fy_out) Fy_out[c] = Fy;
    if (p_out) p_out[c] = rho[c] * CS2;
  }
}

void vo_macroscopic(const vo_params *P, const double *phi,
                    const unsigned char *mask, const double *fext_x,
                    const double *fext_y, const double *f, double *m0_out,
                    double *rho_out, double *ux_out, double *uy_out,
                    double *Fx_out, double *Fy_out, double *p_out) {
  vo_nbr T;
  vo_work W;
  if (work_alloc(P->nx * P->ny, &W) != 0) return;
  if (nbr_build(P, mask, &T) == 0)
    macroscopic_tab(P, &T, &W, phi, mask, fext_x, fext_y, f, m0_out, rho_out,
                    ux_out, uy_out, Fx_out, Fy_out, p_out);
  nbr_free(&T);
  work_free(&W);
}

static void feq_of(const vo_params *P, double phi, double rho, double ux,
                   double uy, double *feq);

/* ---- one time step, Eq. (16) followed by streaming ------------------------
 * f: post-stream populations at t; fout receives those at t+1.  phi_next,
 * mask, fext_x, fext_y may be NULL.  Returns 0, or -1 on allocation failure. */
static int step_tab(const vo_params *P, const vo_nbr *Tp, vo_work *W,
                    const double *phi, const double *phi_next,
                    const unsigned char *mask, const double *fext_x,
                    const double *fext_y, const double *f, double *fout) {
  const int nx = P->nx, ny = P->ny, N = nx * ny;
  double *m0 = W->m0, *rho = W->rho, *ux = W->ux, *uy = W->uy, *Fx = W->Fx,
         *Fy = W->Fy;
  /* product fields and their eight derivatives (O4-O5) */
  double *rux = W->rux, *ruy = W->ruy, *mux = W->mux, *muy = W->muy, *d = W->d,
         *tmp = W->tmp;
  double *d_rux_x = d, *d_ruy_y = d + N, *d_ux_x = d + 2 * (size_t)N,
         *d_uy_y = d + 3 * (size_t)N, *d_uy_x = d + 4 * (size_t)N,
         *d_ux_y = d + 5 * (size_t)N, *d_mux_x = d + 6 * (size_t)N,
         *d_muy_y = d + 7 * (size_t)N, *d_ruy_x = d + 8 * (size_t)N,
         *d_rux_y = d + 9 * (size_t)N, *d_muy_x = d + 10 * (size_t)N,
         *d_mux_y = d + 11 * (size_t)N;

  const vo_nbr T = *Tp;

  /* O1-O3: rho, F = F^p + F^B, u (Eq. 7, Eq. 13) */
  macroscopic_tab(P, &T, W, phi, mask, fext_x, fext_y, f, m0, rho, ux, uy, Fx,
                  Fy, NULL);

  /* O4: node-wise product fields */
#pragma omp parallel for schedule(static)
  for (int c = 0; c < N; ++c) {
    rux[c] = rho[c] * ux[c];
    ruy[c] = rho[c] * uy[c];
    mux[c] = m0[c] * ux[c]; /* phi*rho*u_x with phi*rho = sum_i f_i */
    muy[c] = m0[c] * uy[c];
  }

  /* O5: the eight derivatives of Eq. (20), each by Eq. (10) */
  gradient_wall(P, mask, &T, rux, 1, 1, rho, d_rux_x, d_rux_y);
  gradient_wall(P, mask, &T, ruy, 1, 0, NULL, d_ruy_x, d_ruy_y);
  gradient_wall(P, mask, &T, ux, 1, 1, NULL, d_ux_x, d_ux_y);
  gradient_wall(P, mask, &T, uy, 1, 0, NULL, d_uy_x, d_uy_y);
  gradient_wall(P, mask, &T, mux, 1, 1, m0, d_mux_x, d_mux_y);
  gradient_wall(P, mask, &T, muy, 1, 0, NULL, d_muy_x, d_muy_y);
  (void)tmp;

  const double s[9] = {P->s_c, P->s_e, P->s_eps, P->s_c, P->s_q,
                       P->s_c, P->s_q, P->s_nu, P->s_nu};

  double *fpost = W->fp;

  /* O6-O9 at every fluid node */
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const int c = y * nx + x;
      if (is_solid(mask, c) || nee_row(P, y)) continue;

      /* O6: penalty source C = (0, C_a, 0, 0, 0, 0, 0, C_b, C_c), Eq. (20) */
      const double dt_phi = phi_next ? (phi_next[c] - phi[c]) : 0.0;
      const double dd[12] = {d_rux_x[c], d_ruy_y[c], d_ux_x[c], d_uy_y[c],
                             d_uy_x[c],  d_ux_y[c],  d_mux_x[c], d_muy_y[c],
                             d_ruy_x[c], d_rux_y[c], d_muy_x[c], d_mux_y[c]};
      const double kmp = P->kappa - (P->model_b ? 1.0 : phi[c]);
      double Cabc[3];
      if (P->eq2)
        vo_penalty_b3(phi[c], rho[c], P->kappa, kmp, dt_phi, dd, Cabc);
      else
        penalty20(phi[c], rho[c], P->kappa, kmp, dt_phi, dd, Cabc);
      double C[9] = {0, Cabc[0], 0, 0, 0, 0, 0, Cabc[1], Cabc[2]};
      if (!P->use_penalty)
        for (int k = 0; k < 9; ++k) C[k] = 0.0;

      /* O7: m = M f (Eq. 17), m^eq (Eq. 18), S (Eq. 19) */
      double fl[9], m[9], meq[9], S[9], mp[9];
      for (int i = 0; i < 9; ++i) fl[i] = f[(size_t)i * N + c];
      for (int k = 0; k < 9; ++k) {
        double acc = 0.0;
        for (int i = 0; i < 9; ++i) acc += MM[k][i] * fl[i];
        m[k] = acc;
      }
      if (P->eq2)
        vo_meq2(phi[c], rho[c], ux[c], uy[c], P->kappa, meq);
      else
        vo_meq(phi[c], rho[c], ux[c], uy[c], P->kappa, meq);
      vo_force_moments(ux[c], uy[c], Fx[c], Fy[c], S);

      /* O8: m+ = m - Gamma (m - m^eq) + (I - Gamma/2)(S + C), Eq. (16) */
      for (int k = 0; k < 9; ++k)
        mp[k] = m[k] - s[k] * (m[k] - meq[k]) + (1.0 - 0.5 * s[k]) * (S[k] + C[k]);

      /* O9: f+ = M^-1 m+ (Eq. A1) */
      for (int i = 0; i < 9; ++i) {
        double acc = 0.0;
        for (int k = 0; k < 9; ++k) acc += MINV36[i][k] * mp[k];
        fpost[(size_t)i * N + c] = acc / 36.0;
      }
    }

  /* Velocity boundary rows (non-equilibrium extrapolation, Sec. 3.1):
   * f+(x_b) = f^eq(phi(x_b), rho(x_f), u_w) + f+(x_f) - f^eq(phi(x_f), rho(x_f), u(x_f)) */
  for (int y = 0; y < ny; ++y) {
    const int kind = nee_row(P, y);
    if (!kind) continue;
    const int yf = (kind == 1) ? 1 : ny - 2;
    const double uw = (kind == 1) ? P->un_lo : P->un_hi;
    for (int x = 0; x < nx; ++x) {
      const int c = y * nx + x, cf = yf * nx + x;
      double eb[9], ef[9];
      feq_of(P, phi[c], rho[cf], uw, 0.0, eb);
      feq_of(P, phi[cf], rho[cf], ux[cf], uy[cf], ef);
      for (int i = 0; i < 9; ++i)
        fpost[(size_t)i * N + c] = eb[i] + (fpost[(size_t)i * N + cf] - ef[i]);
    }
  }

#pragma omp parallel for schedule(static)
  for (long k = 0; k < 9L * N; ++k) fout[k] = 0.0;

  /* O10: push streaming f_i(x+e_i, t+1) = f+_i(x, t); half-way bounce-back
   * off walls and solid nodes: f_opp(i)(x, t+1) = f+_i(x, t).  Every (target
   * node, direction) of fout is written by exactly one source. */
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const int c = y * nx + x;
      if (is_solid(mask, c)) continue;
      double fp[9];
      for (int i = 0; i < 9; ++i) fp[i] = fpost[(size_t)i * N + c];
      for (int i = 0; i < 9; ++i) {
        int xn = x + EX[i], yn = y + EY[i];
        int blocked = 0;
        double uw = 0.0; /* tangential velocity of the wall crossed */
        if (xn < 0 || xn >= nx) {
          if (P->bc_x == 0) xn = (xn + nx) % nx; else blocked = 1;
        }
        if (yn < 0 || yn >= ny) {
          if (P->bc_y == 0) {
            yn = (yn + ny) % ny;
          } else {
            blocked = 1;
            uw = (yn < 0) ? P->uw_lo : P->uw_hi;
          }
        }
        if (!blocked && is_solid(mask, yn * nx + xn)) blocked = 1;
        if (blocked && uw != 0.0) {
          /* moving wall: subtract the odd part of the equilibrium at u_w */
          double fw[9];
          feq_of(P, phi[c], P->rho_w, uw, 0.0, fw);
          fout[(size_t)OPP[i] * N + c] = fp[i] - (fw[i] - fw[OPP[i]]);
        } else if (blocked)
          fout[(size_t)OPP[i] * N + c] = fp[i];
        else
          fout[(size_t)i * N + (yn * nx + xn)] = fp[i];
      }
    }

  return 0;
}

int vo_step(const vo_params *P, const double *phi, const double *phi_next,
            const unsigned char *mask, const double *fext_x,
            const double *fext_y, const double *f, double *fout) {
  vo_nbr T;
  vo_work W;
  if (work_alloc(P->nx * P->ny, &W) != 0) return -1;
  if (nbr_build(P, mask, &T) != 0) {
    work_free(&W);
    return -1;
  }
  const int rc = step_tab(P, &T, &W, phi, phi_next, mask, fext_x, fext_y, f, fout);
  nbr_free(&T);
  work_free(&W);
  return rc;
}

/* Second-order truncated equilibrium of Appendix B, Eq. (B1). */
void vo_feq2(double phi, double rho, double ux, double uy, double kappa,
             double *feq) {
  const double uu = ux * ux + uy * uy;
  double sum_w_nonzero = 0.0;
  for (int i = 1; i < 9; ++i) sum_w_nonzero += WT[i];
  feq[0] = phi * rho - sum_w_nonzero * kappa * rho -
           WT[0] * phi * rho * uu / (2.0 * CS2);
  for (int i = 1; i < 9; ++i) {
    const double eu = EX[i] * ux + EY[i] * uy;
    feq[i] = WT[i] * (kappa * rho + phi * rho * (eu / CS2 + eu * eu / (2.0 * CS2 * CS2) -
                                                 uu / (2.0 * CS2)));
  }
}

/* The equilibrium the scheme relaxes to: Eq. (14), or (B1) with eq2. */
static void feq_of(const vo_params *P, double phi, double rho, double ux,
                   double uy, double *feq) {
  if (P->eq2)
    vo_feq2(phi, rho, ux, uy, P->kappa, feq);
  else
    vo_feq(phi, rho, ux, uy, P->kappa, feq);
}

/* Initial populations f(0) = f^eq(rho0, u0) of Eq. (14) (or B1) at every
 * fluid node. */
void vo_init_equilibrium(const vo_params *P, const double *phi,
                         const unsigned char *mask, double rho0, double ux0,
                         double uy0, double *f) {
  const int N = P->nx * P->ny;
  for (int c = 0; c < N; ++c) {
    double feq[9] = {0};
    if (!is_solid(mask, c)) feq_of(P, phi[c], rho0, ux0, uy0, feq);
    for (int i = 0; i < 9; ++i) f[(size_t)i * N + c] = feq[i];
  }
}

/* Same with a per-node density and velocity (used to start shear waves,
 * manufactured solutions and random states). */
void vo_init_fields(const vo_params *P, const double *phi,
                    const unsigned char *mask, const double *rho,
                    const double *ux, const double *uy, double *f) {
  const int N = P->nx * P->ny;
  for (int c = 0; c < N; ++c) {
    double feq[9] = {0};
    if (!is_solid(mask, c)) feq_of(P, phi[c], rho[c], ux[c], uy[c], feq);
    for (int i = 0; i < 9; ++i) f[(size_t)i * N + c] = feq[i];
  }
}

/* n steps in a row with static phi and forcing; f is updated in place. */
int vo_run(const vo_params *P, const double *phi, const unsigned char *mask,
           const double *fext_x, const double *fext_y, double *f, long nsteps) {
  const size_t n9 = (size_t)9 * P->nx * P->ny;
  double *g = malloc(n9 * sizeof(double));
  vo_nbr T;
  vo_work W;
  if (!g || work_alloc(P->nx * P->ny, &W) != 0) {
    free(g);
    return -1;
  }
  if (nbr_build(P, mask, &T) != 0) {
    work_free(&W);
    free(g);
    return -1;
  }
  int rc = 0;
  double *a = f, *b = g; /* alternate the two arrays; the result ends in f */
  for (long t = 0; t < nsteps && rc == 0; ++t) {
    rc = step_tab(P, &T, &W, phi, NULL, mask, fext_x, fext_y, a, b);
    double *tmp = a; a = b; b = tmp;
  }
  if (rc == 0 && a != f) memcpy(f, a, n9 * sizeof(double));
  nbr_free(&T);
  work_free(&W);
  free(g);
  return rc;
}
