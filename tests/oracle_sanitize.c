/* Driver that runs the FP64 oracle (compiled into this translation unit)
 * under AddressSanitizer and UndefinedBehaviorSanitizer: every boundary type
 * and optional input on small, ragged lattices, so an out-of-bounds index or
 * an undefined operation anywhere in the oracle aborts the run.  Built and
 * run by tests/test_oracle_sanitize.py; exit code 0 when every result is
 * finite. */
#include "../oracle/vanse_oracle.c"

#include <stdio.h>

static unsigned long long lcg = 12345;
static double urand(void) {
  lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
  return (double)(lcg >> 11) / 9007199254740992.0;
}

static int finite_all(const double *a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(a[i])) return 0;
  return 1;
}

static vo_params params(int nx, int ny, int bc_y) {
  vo_params P;
  memset(&P, 0, sizeof P);
  P.nx = nx;
  P.ny = ny;
  P.bc_x = 0;
  P.bc_y = bc_y;
  P.kappa = 0.5;
  P.s_c = 1.0;
  P.s_e = 1.2;
  P.s_eps = 1.2;
  P.s_q = 1.2;
  P.s_nu = 0.8;
  P.gx = 1e-5;
  P.gy = -2e-6;
  P.scale_by_phi = 1;
  P.use_penalty = 1;
  P.rho_w = 1.0;
  return P;
}

/* One case: n steps with vo_run, one with vo_step (phi_next given), and the
 * read-outs; returns 0 when everything stays finite. */
static int run_case(const char *name, vo_params P, int with_mask, int with_force,
                    int with_drag) {
  const int N = P.nx * P.ny;
  double *phi = malloc(sizeof(double) * N), *phin = malloc(sizeof(double) * N);
  double *fx = malloc(sizeof(double) * N), *fy = malloc(sizeof(double) * N);
  double *beta = malloc(sizeof(double) * N);
  double *f = malloc(sizeof(double) * 9 * N), *g = malloc(sizeof(double) * 9 * N);
  double *out[7];
  for (int k = 0; k < 7; ++k) out[k] = malloc(sizeof(double) * N);
  unsigned char *mask = malloc(N);
  for (int c = 0; c < N; ++c) {
    phi[c] = 0.5 + 0.45 * urand();
    phin[c] = phi[c] * (1.0 + 1e-3 * (urand() - 0.5));
    fx[c] = 1e-6 * (urand() - 0.5);
    fy[c] = 1e-6 * (urand() - 0.5);
    beta[c] = 1e-3 + 1e-2 * urand();
    mask[c] = (urand() < 0.1) ? 1 : 0;
  }
  /* solid nodes on the first and last columns and rows as well */
  if (with_mask) {
    mask[0] = mask[N - 1] = mask[P.nx - 1] = mask[N - P.nx] = 1;
  }
  const unsigned char *m = with_mask ? mask : NULL;
  if (with_drag) {
    P.beta = beta;
    P.usx = 1e-4;
  }
  vo_init_equilibrium(&P, phi, m, 1.0, 1e-3, -5e-4, f);
  int rc = vo_run(&P, phi, m, with_force ? fx : NULL, with_force ? fy : NULL, f, 5);
  if (rc == 0) rc = vo_step(&P, phi, phin, m, with_force ? fx : NULL, with_force ? fy : NULL, f, g);
  if (rc == 0) {
    vo_macroscopic(&P, phin, m, with_force ? fx : NULL, with_force ? fy : NULL, g, out[0], out[1],
                   out[2], out[3], out[4], out[5], out[6]);
    vo_gradient(&P, m, out[1], 0, out[4], out[5]);
    vo_gradient(&P, m, out[2], 1, out[4], out[5]);
  }
  int ok = rc == 0 && finite_all(g, (size_t)9 * N);
  for (int k = 0; k < 7 && ok; ++k) ok = finite_all(out[k], N);
  printf("%-40s %s\n", name, ok ? "ok" : "FAILED");
  free(phi); free(phin); free(fx); free(fy); free(beta); free(f); free(g); free(mask);
  for (int k = 0; k < 7; ++k) free(out[k]);
  return ok ? 0 : 1;
}

int main(void) {
  int bad = 0;
  bad |= run_case("periodic 13x11", params(13, 11, 0), 0, 0, 0);
  bad |= run_case("walls 17x9, force field, drag", params(17, 9, 1), 0, 1, 1);
  bad |= run_case("walls 10x7, mask", params(10, 7, 1), 1, 0, 0);
  bad |= run_case("periodic 3x5, mask, force field", params(3, 5, 0), 1, 1, 0);
  {
    vo_params P = params(12, 8, 1);
    P.model_b = 1;
    P.eq2 = 1;
    P.uw_lo = 1e-3;
    P.uw_hi = -2e-3;
    bad |= run_case("walls 12x8, model B, App. B, moving walls", P, 1, 1, 1);
  }
  {
    vo_params P = params(11, 7, 1);
    P.bc_x = 1;
    P.uw_hi = 2e-3;
    bad |= run_case("box 11x7, walls in x, mask, force field, drag, lid", P, 1, 1, 1);
  }
  {
    vo_params P = params(5, 9, 0);
    P.bc_x = 1;
    bad |= run_case("walls in x 5x9, periodic in y, mask", P, 1, 0, 0);
  }
  {
    vo_params P = params(10, 3, 1);
    P.nee_lo = P.nee_hi = 1;
    P.un_lo = -1e-3;
    P.un_hi = 2e-3;
    bad |= run_case("walls 10x3, velocity rows on both faces, drag", P, 0, 1, 1);
  }
  {
    vo_params P = params(7, 9, 1);
    P.eq2 = 1;
    P.nee_hi = 1;
    P.un_hi = 1e-3;
    bad |= run_case("walls 7x9, App. B, upper velocity row", P, 0, 0, 0);
  }
  {
    vo_params P = params(9, 6, 1);
    P.use_penalty = 0;
    P.scale_by_phi = 0;
    bad |= run_case("walls 9x6, no penalty, F^B = G", P, 0, 0, 0);
  }
  return bad;
}
