/*
 * psc_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU reference for the per-time-step
 * partially-saturated-cell (PSC) lattice Boltzmann update of Liu & Wu,
 * "A hybrid LBM-DEM framework with an improved immersed moving boundary
 * method for modelling complex particle-liquid flows involving adhesive
 * particles" (arXiv 1901.09745), plus its adhesive (JKR) DEM step.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code, header, table or helper with the
 * HIP library; the velocity sets below are written out here independently.
 *
 * Layout: f is stored "natural" and canonical, f[i][z][y][x] in FP64, with the
 * velocity order
 *   D2Q9 : 0 (0,0) 1 (1,0) 2 (0,1) 3 (-1,0) 4 (0,-1) 5 (1,1) 6 (-1,1)
 *          7 (-1,-1) 8 (1,-1)
 *   D3Q19: 0 rest, 1/2 = +-x, 3/4 = +-y, 5/6 = +-z, then the 12 edge vectors
 *          in (v, -v) pairs: xy(++,--), xy(+-,-+), xz(++,--), xz(+-,-+),
 *          yz(++,--), yz(+-,-+).
 * Cell n = x + nx*(y + ny*z) has its centre at the integer point (x, y, z) and
 * covers [x-1/2, x+1/2] along each axis.
 *
 * Every step below is written in the order the paper gives it:
 *   Sec. 2.1 Eqs. 1-5 (BGK + Guo forcing), Sec. 2.2 Eq. 6 (bounce-back),
 *   Sec. 2.3 Eqs. 10, 12-14 (modified PSC collision and per-particle forces),
 *   Sec. 2.4 Eqs. 15-19 and Table 1 (linear solid fraction),
 *   Sec. 2.5 Eqs. 21, 25-27 (Newton-Euler motion with the JKR normal force,
 *   or Hertz's without adhesion) and Eqs. 22, 28, 29 (sliding, twisting and
 *   rolling friction, optional).
 * Readings of points the paper leaves open are marked "Reading:".
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Velocity sets (textbook D2Q9; D3Q19 weights 1/3, 1/18, 1/36 per Eq. 3).   */
/* ------------------------------------------------------------------------ */
static const int E9[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double W9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const int E19[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double W19[19] = {
    1.0 / 3,
    1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

#define OR_QMAX 19
#define OR_KMAX 16 /* particles recorded per cell by the oracle */

/* Face boundary kinds.  Faces: 0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+. */
enum { OR_PERIODIC = 0, OR_BOUNCE_BACK = 1, OR_MOVING_WALL = 2,
       OR_INLET_EQ = 3, OR_OUTLET_EQ = 4 };

typedef struct {
  int q;              /* 9 or 19 */
  int nx, ny, nz;     /* nz == 1 for D2Q9 */
  double tau;         /* relaxation time (lattice units) */
  double force[3];    /* constant body-force density on the fluid */
  int face_bc[6];     /* per face kind (see enum) */
  double face_u[6][3];/* wall velocity (MOVING_WALL) / inlet velocity (INLET_EQ) */
  double rho0;        /* reference density (inlet / outlet density) */
  double h;           /* half-width of the solid-fraction shell (Sec. 2.4) */
} or_config;

typedef struct {
  double rho_p, rho_f; /* particle and fluid densities */
  double E_p, poisson; /* particle Young modulus and Poisson ratio (Eq. 25) */
  double gamma;        /* surface energy (Eq. 27) */
  double eta_n;        /* normal damping coefficient (Eq. 26) */
  double g[3];         /* gravitational acceleration */
  double dt;           /* coupling time step (one LBM step) */
  int n_sub;           /* DEM sub-cycles per coupling step (ratio lambda) */
  int kinematic;       /* 1: X += dt*U only (prescribed motion) */
  double k_t;          /* tangential stiffness k_T (Eq. 28) */
  double eta_t;        /* tangential dissipation coefficient eta_T (Eq. 28) */
  double mu_f;         /* friction coefficient (Eq. 29); 0: no sliding or twisting friction */
  double theta_r;      /* critical rolling angle theta_crit (Eq. 29); 0: no rolling resistance */
} or_dem_params;

int or_version(void) { return 1; }

static int lat_q(const or_config* c) { return c->q; }
static int ex(int q, int i, int a) { return q == 9 ? E9[i][a] : E19[i][a]; }
static double wt(int q, int i) { return q == 9 ? W9[i] : W19[i]; }
static int opp(int q, int i) {
  for (int j = 0; j < q; ++j)
    if (ex(q, j, 0) == -ex(q, i, 0) && ex(q, j, 1) == -ex(q, i, 1) &&
        ex(q, j, 2) == -ex(q, i, 2))
      return j;
  return -1;
}
static int dims(const or_config* c, int a) {
  return a == 0 ? c->nx : (a == 1 ? c->ny : c->nz);
}
/* An axis is periodic when both of its faces are periodic; the z axis of a
 * D2Q9 lattice (nz == 1) is treated as periodic. */
static int axis_periodic(const or_config* c, int a) {
  if (a == 2 && c->q == 9) return 1;
  return c->face_bc[2 * a] == OR_PERIODIC && c->face_bc[2 * a + 1] == OR_PERIODIC;
}

/* Minimum-image separation along one axis (Reading: periodic distances and
 * torque arms use the nearest image). */
static double min_image(const or_config* c, int a, double d) {
  if (!axis_periodic(c, a)) return d;
  double L = (double)dims(c, a);
  if (d > 0.5 * L) d -= L;
  else if (d < -0.5 * L) d += L;
  return d;
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.4: linear solid-fraction approximation                             */
/* ------------------------------------------------------------------------ */

/* Eq. 19: V_a in 2D, the integral of sqrt(r^2 - x^2) over [-1/2, 1/2]. */
double or_va2d(double r) {
  double s = sqrt(r * r - 0.25);
  return 0.5 * s + r * r * atan(0.5 / s);
}

/* Eq. 17: V_a in 3D, the integral of sqrt(r^2 - x^2 - y^2) over the unit
 * square.  Reading: the printed integrand lacks its square root (the closed
 * form is the integral of the root); the first arctangent is the principal
 * value even though its denominator 1/2 - r^2 is negative. */
double or_va3d(double r) {
  double r2 = r * r;
  double s = sqrt(r2 - 0.5);
  return (1.0 / 12.0 - r2) * atan(0.5 * s / (0.5 - r2)) + s / 3.0 +
         (r2 - 1.0 / 12.0) * atan(0.5 / s) -
         (4.0 / 3.0) * r2 * r * atan(0.25 / (r * s));
}

/* Eq. 18 with Eq. 15 and D = d - r: eps = -D + f(r) = V_a(r) + 1/2 - d. */
static double linear_eps_offset(int q, double r) {
  return (q == 9 ? or_va2d(r) : or_va3d(r)) + 0.5;
}

/* Fraction of a cell covered by a particle (Sec. 2.4).  With the gap D = d - r
 * between the cell centre and the particle surface, Eqs. 15 and 18 reduce the
 * linear approximation to eps = V_a(r) + 1/2 - d (cs = V_a(r) + 1/2), which is
 * kept within [0, 1].  The text applies the formula to the shell of half-width
 * h about the surface only: a cell centre at least r + h from the particle
 * centre lies outside (0), one at most r - h from it inside (1).  Reading:
 * Table 1 prints these two values the other way round; the text is followed. */
static double cell_fraction(double d, double r, double h, double cs) {
  if (d >= r + h) return 0.0;
  if (d <= r - h) return 1.0;
  double eps = cs - d;
  if (eps <= 0.0) return 0.0;
  if (eps >= 1.0) return 1.0;
  return eps;
}

/* Lattice index of the cell at integer position k (nearest image on periodic
 * axes); -1 when k lies beyond a walled axis. */
static int cell_at(const or_config* c, const int* k) {
  int p[3];
  for (int a = 0; a < 3; ++a) {
    int L = dims(c, a);
    if (axis_periodic(c, a)) p[a] = ((k[a] % L) + L) % L;
    else if (k[a] < 0 || k[a] >= L) return -1;
    else p[a] = k[a];
  }
  return p[0] + c->nx * (p[1] + c->ny * p[2]);
}

/* Solid fractions of all particles (Sec. 2.4, Eqs. 15-19).  Every cell whose
 * fraction can be nonzero has its centre within r + h of the particle centre
 * along each axis, so those cells are the candidates examined.  Each cell n
 * gets the list of particles covering it with eps_{n,s} > 0 (nslot[n] of them,
 * ids in slot_id[n*kmax ..] in ascending order, fractions in slot_eps) and the
 * unclamped total eps_sum[n] = sum_s eps_{n,s}; the clamp of the total at one
 * is taken where the total is used (or_weights).  Returns 0, or -1 when a cell
 * is covered by more than kmax particles, -2 on a radius outside the domain of
 * Eqs. 17/19. */
int or_rasterize(const or_config* c, int np, const double* X, const double* R,
                 int kmax, int* nslot, int* slot_id, double* slot_eps,
                 double* eps_sum) {
  const int q = lat_q(c);
  const int N = c->nx * c->ny * c->nz;
  const int dim = q == 9 ? 2 : 3;
  const double h = c->h;
  for (int n = 0; n < N; ++n) { nslot[n] = 0; eps_sum[n] = 0.0; }
  for (int s = 0; s < np; ++s) {
    const double r = R[s];
    if (!(r * r > (q == 9 ? 0.25 : 0.5))) return -2;
    const double cs = linear_eps_offset(q, r);
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
      lo[a] = (int)ceil(X[3 * s + a] - (r + h));
      hi[a] = (int)floor(X[3 * s + a] + (r + h));
    }
    int k[3];
    for (k[2] = lo[2]; k[2] <= hi[2]; ++k[2])
      for (k[1] = lo[1]; k[1] <= hi[1]; ++k[1])
        for (k[0] = lo[0]; k[0] <= hi[0]; ++k[0]) {
          const int n = cell_at(c, k);
          if (n < 0) continue;
          /* centre-to-centre distance d, nearest image */
          const int p[3] = {n % c->nx, (n / c->nx) % c->ny, n / (c->nx * c->ny)};
          double d2 = 0.0;
          for (int a = 0; a < dim; ++a) {
            double dx = min_image(c, a, (double)p[a] - X[3 * s + a]);
            d2 += dx * dx;
          }
          const double eps = cell_fraction(sqrt(d2), r, h, cs);
          if (!(eps > 0.0)) continue;
          if (nslot[n] >= kmax) return -1;
          slot_id[n * kmax + nslot[n]] = s;
          slot_eps[n * kmax + nslot[n]] = eps;
          nslot[n] += 1;
          eps_sum[n] += eps;
        }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.1: equilibrium, forcing and moments                                */
/* ------------------------------------------------------------------------ */

/* Eq. 3 with c_s^2 = 1/3. */
void or_feq(int q, double rho, const double* u, double* out) {
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < q; ++i) {
    double eu = ex(q, i, 0) * u[0] + ex(q, i, 1) * u[1] + ex(q, i, 2) * u[2];
    out[i] = rho * wt(q, i) * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
  }
}

/* Eq. 4: F_i = (1 - 1/(2 tau)) w_i [ (e_i - u)/c_s^2 + (e_i.u) e_i / c_s^4 ] . F */
void or_guo(int q, double tau, const double* u, const double* F, double* out) {
  for (int i = 0; i < q; ++i) {
    double eu = ex(q, i, 0) * u[0] + ex(q, i, 1) * u[1] + ex(q, i, 2) * u[2];
    double s = 0.0;
    for (int a = 0; a < 3; ++a)
      s += (3.0 * (ex(q, i, a) - u[a]) + 9.0 * eu * ex(q, i, a)) * F[a];
    out[i] = (1.0 - 1.0 / (2.0 * tau)) * wt(q, i) * s;
  }
}

/* Eq. 5: rho = sum f, rho u = sum f e + F/2 (unit time step). */
void or_moments(int q, const double* f, const double* F, double* rho, double* u) {
  double m = 0.0, j[3] = {0, 0, 0};
  for (int i = 0; i < q; ++i) {
    m += f[i];
    for (int a = 0; a < 3; ++a) j[a] += f[i] * ex(q, i, a);
  }
  *rho = m;
  for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * F[a]) / m;
}

/* Eq. 10: Omega^s_i = f_{-i} - f^eq_{-i}(rho, u) + f^eq_i(rho, u_s) - f_i. */
void or_omega_s(int q, const double* f, double rho, const double* u,
                const double* us, double* out) {
  double fe[OR_QMAX], fs[OR_QMAX];
  or_feq(q, rho, u, fe);
  or_feq(q, rho, us, fs);
  for (int i = 0; i < q; ++i) {
    int o = opp(q, i);
    out[i] = f[o] - fe[o] + fs[i] - f[i];
  }
}

/* Weighting functions of Sec. 2.3.
 * mode 0 (the paper's modified scheme): eps_n = min(sum eps, 1) (the
 *   clamped cell total of Sec. 2.4) and Eq. 13, B_{n,s} = eps_{n,s}(tau-1/2)/((1-eps_n)+tau-1/2);
 *   B_n = eps_n(tau-1/2)/((1-eps_n)+tau-1/2), which is the sum of the B_{n,s}.
 *   Reading: when the recorded fractions sum above one the total is clamped
 *   to 1 (B_n = 1) and each particle keeps its share, B_{n,s} = eps_{n,s}/sum,
 *   so that the shares still add up to B_n.
 * mode 1 (the original scheme, Eqs. 8-9): B_{n,s} from Eq. 9 per particle and
 *   B_n = sum_s B_{n,s}. */
void or_weights(int nslot, const double* eps, double tau, int mode,
                double* B_total, double* B_slot) {
  double S = 0.0;
  for (int k = 0; k < nslot; ++k) S += eps[k];
  double tm = tau - 0.5;
  if (mode == 1) {
    double B = 0.0;
    for (int k = 0; k < nslot; ++k) {
      B_slot[k] = eps[k] * tm / ((1.0 - eps[k]) + tm);
      B += B_slot[k];
    }
    *B_total = B;
    return;
  }
  double en = S < 1.0 ? S : 1.0;
  *B_total = en * tm / ((1.0 - en) + tm);
  for (int k = 0; k < nslot; ++k)
    B_slot[k] = (S <= 1.0) ? eps[k] * tm / ((1.0 - en) + tm) : eps[k] / S;
}

/* ------------------------------------------------------------------------ */
/* Boundary layers with prescribed equilibrium (inlet / outlet)              */
/* ------------------------------------------------------------------------ */
/* Reading (the paper names a constant-velocity inlet and a constant-pressure
 * outlet in Sec. 3.2 without a scheme): before each collision the cells of an
 * INLET_EQ face layer take f = f^eq(rho0, u_face) and the cells of an
 * OUTLET_EQ face layer take f = f^eq(rho0, u), u being the Eq. 5 velocity of
 * the adjacent interior cell (zero normal gradient) at the same time level.
 * Outlet layers are resolved first (from the unmodified state), then inlet
 * layers.  Links that leave the domain through such a face are reflected like
 * a resting wall; the reflected values are overwritten by this reset.
 * Open faces need at least three cells across their axis. */
static void apply_open_layers(const or_config* c, double* f) {
  const int q = lat_q(c), N = c->nx * c->ny * c->nz;
  /* Every outlet cell takes the velocity of its interior neighbour in the
   * state entering the step, before any layer is reset (where two outlet
   * faces meet, the neighbour may itself be an outlet cell); a cell on two
   * outlet faces takes the later face's neighbour. */
  double* ub = NULL;
  int* has = NULL;
  int any_outlet = 0;
  for (int face = 0; face < 6; ++face) any_outlet |= c->face_bc[face] == OR_OUTLET_EQ;
  if (any_outlet) {
    ub = (double*)calloc((size_t)3 * N, sizeof(double));
    has = (int*)calloc((size_t)N, sizeof(int));
    for (int face = 0; face < 6; ++face) {
      if (c->face_bc[face] != OR_OUTLET_EQ) continue;
      int a = face / 2, L = dims(c, a);
      int layer = (face % 2 == 0) ? 0 : L - 1;
      int inward = (face % 2 == 0) ? 1 : -1;
      for (int z = 0; z < c->nz; ++z)
        for (int y = 0; y < c->ny; ++y)
          for (int x = 0; x < c->nx; ++x) {
            int p[3] = {x, y, z};
            if (p[a] != layer) continue;
            int n = x + c->nx * (y + c->ny * z);
            int pn[3] = {x, y, z};
            pn[a] += inward;
            int m = pn[0] + c->nx * (pn[1] + c->ny * pn[2]);
            double fl[OR_QMAX], rho;
            for (int i = 0; i < q; ++i) fl[i] = f[(size_t)i * N + m];
            or_moments(q, fl, c->force, &rho, &ub[3 * (size_t)n]);
            has[n] = 1;
          }
    }
    for (int n = 0; n < N; ++n) {
      if (!has[n]) continue;
      double fe[OR_QMAX];
      or_feq(q, c->rho0, &ub[3 * (size_t)n], fe);
      for (int i = 0; i < q; ++i) f[(size_t)i * N + n] = fe[i];
    }
    free(ub);
    free(has);
  }
  /* inlets afterwards: an inlet face wins where it meets an outlet */
  for (int face = 0; face < 6; ++face) {
    if (c->face_bc[face] != OR_INLET_EQ) continue;
    int a = face / 2, L = dims(c, a);
    int layer = (face % 2 == 0) ? 0 : L - 1;
    double fe[OR_QMAX];
    or_feq(q, c->rho0, c->face_u[face], fe);
    for (int z = 0; z < c->nz; ++z)
      for (int y = 0; y < c->ny; ++y)
        for (int x = 0; x < c->nx; ++x) {
          int p[3] = {x, y, z};
          if (p[a] != layer) continue;
          int n = x + c->nx * (y + c->ny * z);
          for (int i = 0; i < q; ++i) f[(size_t)i * N + n] = fe[i];
        }
  }
}

/* ------------------------------------------------------------------------ */
/* One PSC-LBM step (Eqs. 1, 6, 10, 12-14)                                   */
/* ------------------------------------------------------------------------ */

/* Solid velocity at the cell centre: u_s = U_s + Omega_s x r_ns (Reading:
 * the rigid-body velocity of particle s at the node). */
static void solid_velocity(const double* U, const double* W, const double* r,
                           double* us) {
  us[0] = U[0] + W[1] * r[2] - W[2] * r[1];
  us[1] = U[1] + W[2] * r[0] - W[0] * r[2];
  us[2] = U[2] + W[0] * r[1] - W[1] * r[0];
}

static void arm(const or_config* c, int n, const double* Xs, double* r) {
  int p[3] = {n % c->nx, (n / c->nx) % c->ny, n / (c->nx * c->ny)};
  for (int a = 0; a < 3; ++a) {
    if (a == 2 && c->q == 9) { r[a] = 0.0; continue; }
    r[a] = min_image(c, a, (double)p[a] - Xs[a]);
  }
}

/* One time step on the natural-layout FP64 state f[Q][N] (in place).
 * mode: 0 = modified weighting (Eqs. 12-14), 1 = original (Eqs. 7-9, 11).
 * F, T (3*np each) receive the hydrodynamic force and torque of Eq. 14 (or
 * Eq. 11) exerted during this step; T is a 3-vector (only z in 2D).
 * Returns 0, or the rasterizer's error code. */
int or_lbm_step(const or_config* c, int mode, double* f, int np,
                const double* X, const double* U, const double* W,
                const double* R, double* F, double* T) {
  const int q = lat_q(c);
  const int N = c->nx * c->ny * c->nz;
  const int K = OR_KMAX;
  const double tau = c->tau;
  int* nslot = (int*)malloc(sizeof(int) * (size_t)N);
  int* sid = (int*)malloc(sizeof(int) * (size_t)N * K);
  double* seps = (double*)malloc(sizeof(double) * (size_t)N * K);
  double* ssum = (double*)malloc(sizeof(double) * (size_t)N);
  double* fn = (double*)malloc(sizeof(double) * (size_t)N * q);
  int rc = 0;
  if (!nslot || !sid || !seps || !ssum || !fn) { rc = -3; goto done; }

  apply_open_layers(c, f);
  rc = or_rasterize(c, np, X, R, K, nslot, sid, seps, ssum);
  if (rc) goto done;

#pragma omp parallel for schedule(static) if (N > 8192)
  for (int n = 0; n < N; ++n) {
    double fl[OR_QMAX], fe[OR_QMAX], Fi[OR_QMAX], fs[OR_QMAX], om[OR_QMAX];
    double rho, u[3];
    for (int i = 0; i < q; ++i) fl[i] = f[(size_t)i * N + n];
    or_moments(q, fl, c->force, &rho, u);          /* Eq. 5 */
    or_feq(q, rho, u, fe);                          /* Eq. 3 */
    or_guo(q, tau, u, c->force, Fi);                /* Eq. 4 */
    double Bn = 0.0, Bs[OR_KMAX];
    int ns = nslot[n];
    if (ns > 0) or_weights(ns, &seps[(size_t)n * K], tau, mode, &Bn, Bs);
    /* Eq. 12 (mode 0) / Eq. 7 (mode 1). */
    for (int i = 0; i < q; ++i)
      fs[i] = fl[i] - (1.0 - Bn) * (fl[i] - fe[i]) / tau + (1.0 - Bn) * Fi[i];
    for (int k = 0; k < ns; ++k) {
      int s = sid[(size_t)n * K + k];
      double r[3], us[3];
      arm(c, n, &X[3 * s], r);
      solid_velocity(&U[3 * s], &W[3 * s], r, us);
      or_omega_s(q, fl, rho, u, us, om);            /* Eq. 10 */
      /* Reading for the original scheme with several particles: each
       * particle's operator enters with its own Eq. 9 weight. */
      for (int i = 0; i < q; ++i) fs[i] += Bs[k] * om[i];
    }
    /* Eq. 1 streaming with Eq. 6 bounce-back on walls. */
    int p[3] = {n % c->nx, (n / c->nx) % c->ny, n / (c->nx * c->ny)};
    for (int i = 0; i < q; ++i) {
      int d[3], out = 0;
      double uw[3] = {0, 0, 0};
      for (int a = 0; a < 3; ++a) {
        int L = dims(c, a);
        d[a] = p[a] + ex(q, i, a);
        if (d[a] < 0 || d[a] >= L) {
          if (axis_periodic(c, a)) {
            d[a] = (d[a] + L) % L;
          } else {
            int face = 2 * a + (d[a] < 0 ? 0 : 1);
            out = 1;
            if (c->face_bc[face] == OR_MOVING_WALL)
              for (int b = 0; b < 3; ++b) uw[b] += c->face_u[face][b];
          }
        }
      }
      if (!out) {
        int m = d[0] + c->nx * (d[1] + c->ny * d[2]);
        fn[(size_t)i * N + m] = fs[i];
      } else {
        /* Halfway bounce-back (Eq. 6), with the moving-wall momentum term
         * -2 w_i rho (e_i . u_w) / c_s^2 (Reading: Ladd's moving wall). */
        double eu = ex(q, i, 0) * uw[0] + ex(q, i, 1) * uw[1] + ex(q, i, 2) * uw[2];
        fn[(size_t)opp(q, i) * N + n] = fs[i] - 6.0 * wt(q, i) * rho * eu;
      }
    }
  }

  /* Eq. 14 (mode 0) / Eq. 11 (mode 1): F_s = -sum_n B (sum_i Omega^s_i e_i),
   * T_s = -sum_n r_ns x [B (sum_i Omega^s_i e_i)], over cells in ascending
   * order. */
  for (int s = 0; s < 3 * np; ++s) { F[s] = 0.0; T[s] = 0.0; }
  for (int n = 0; n < N; ++n) {
    int ns = nslot[n];
    if (ns == 0) continue;
    double fl[OR_QMAX], om[OR_QMAX], rho, u[3], Bn, Bs[OR_KMAX];
    for (int i = 0; i < q; ++i) fl[i] = f[(size_t)i * N + n];
    or_moments(q, fl, c->force, &rho, u);
    or_weights(ns, &seps[(size_t)n * K], tau, mode, &Bn, Bs);
    for (int k = 0; k < ns; ++k) {
      int s = sid[(size_t)n * K + k];
      double r[3], us[3], mom[3] = {0, 0, 0};
      arm(c, n, &X[3 * s], r);
      solid_velocity(&U[3 * s], &W[3 * s], r, us);
      or_omega_s(q, fl, rho, u, us, om);
      for (int i = 0; i < q; ++i)
        for (int a = 0; a < 3; ++a) mom[a] += om[i] * ex(q, i, a);
      double B = (mode == 1) ? Bn : Bs[k];
      for (int a = 0; a < 3; ++a) mom[a] *= B;
      for (int a = 0; a < 3; ++a) F[3 * s + a] -= mom[a];
      T[3 * s + 0] -= r[1] * mom[2] - r[2] * mom[1];
      T[3 * s + 1] -= r[2] * mom[0] - r[0] * mom[2];
      T[3 * s + 2] -= r[0] * mom[1] - r[1] * mom[0];
    }
  }
  memcpy(f, fn, sizeof(double) * (size_t)N * q);

done:
  free(nslot); free(sid); free(seps); free(ssum); free(fn);
  return rc;
}

/* f = f^eq(rho[n], u[n]) per cell; rho / u may be NULL (rho0 / rest). */
void or_set_equilibrium(const or_config* c, double* f, const double* rho,
                        const double* u) {
  const int q = lat_q(c), N = c->nx * c->ny * c->nz;
  for (int n = 0; n < N; ++n) {
    double fe[OR_QMAX], uu[3] = {0, 0, 0};
    if (u) for (int a = 0; a < 3; ++a) uu[a] = u[3 * n + a];
    or_feq(q, rho ? rho[n] : c->rho0, uu, fe);
    for (int i = 0; i < q; ++i) f[(size_t)i * N + n] = fe[i];
  }
}

/* Density and velocity fields (Eq. 5) of the state f. */
void or_macros(const or_config* c, const double* f, double* rho, double* u) {
  const int q = lat_q(c), N = c->nx * c->ny * c->nz;
  for (int n = 0; n < N; ++n) {
    double fl[OR_QMAX], r, uu[3];
    for (int i = 0; i < q; ++i) fl[i] = f[(size_t)i * N + n];
    or_moments(q, fl, c->force, &r, uu);
    rho[n] = r;
    for (int a = 0; a < 3; ++a) u[3 * n + a] = uu[a];
  }
}

/* Total mass sum_n sum_i f_i in cell order, with Neumaier's compensated
 * summation so that the result is accurate to about one rounding of the
 * total. */
double or_mass(const or_config* c, const double* f) {
  const int q = lat_q(c), N = c->nx * c->ny * c->nz;
  double s = 0.0, comp = 0.0;
  for (int n = 0; n < N; ++n)
    for (int i = 0; i < q; ++i) {
      double v = f[(size_t)i * N + n];
      double t = s + v;
      if (fabs(s) >= fabs(v)) comp += (s - t) + v;
      else comp += (v - t) + s;
      s = t;
    }
  return s + comp;
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the OpenMP cell loop (timing only; results do not depend on it). */
void or_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.5: JKR adhesive normal contact                                     */
/* ------------------------------------------------------------------------ */
/* Reading (only F_C and a_0 are printed, Eq. 27): with the work of adhesion
 * w = 2 gamma and E from Eq. 25, JKR theory gives, for x = a / a_0,
 *   F / F_C       = 4 (x^3 - x^{3/2})                  (Eq. 26)
 *   delta / delta_C = 6^{1/3} (2 x^2 - (4/3) x^{1/2}),
 *   delta_C       = a_0^2 / (2 6^{1/3} R),
 * where delta = -delta_C at the pull-off point x = 6^{-2/3}.  The paper's
 * pre-computed table of a(delta) is replaced by solving this relation on the
 * stable branch x >= 6^{-2/3} by bisection. */
typedef struct { double FC, a0, dC; } jkr_consts;

static jkr_consts jkr_make(double R, double E, double gamma) {
  jkr_consts k;
  k.FC = 3.0 * M_PI * gamma * R;
  k.a0 = cbrt(9.0 * M_PI * gamma * R * R / E);
  k.dC = k.a0 * k.a0 / (2.0 * cbrt(6.0) * R);
  return k;
}

/* x = a / a0 for a given delta / delta_C >= -1 (stable branch). */
double or_jkr_x(double dn) {
  const double c6 = cbrt(6.0);
  double target = dn / c6;                 /* 2 s^4 - (4/3) s = target */
  double lo = 1.0 / c6;                    /* s = x^{1/2} at pull-off */
  double hi = 1.0;
  while (2.0 * hi * hi * hi * hi - (4.0 / 3.0) * hi < target) hi *= 2.0;
  if (2.0 * lo * lo * lo * lo - (4.0 / 3.0) * lo >= target) return lo * lo;
  for (int it = 0; it < 2000; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (2.0 * mid * mid * mid * mid - (4.0 / 3.0) * mid < target) lo = mid;
    else hi = mid;
  }
  double s = 0.5 * (lo + hi);
  return s * s;
}

/* Effective modulus of two identical bodies (Eq. 25). */
static double eff_modulus(const or_dem_params* p) {
  return 1.0 / (2.0 * (1.0 - p->poisson * p->poisson) / p->E_p);
}

/* Elastic normal contact of effective radius R at overlap delta: the force
 * (repulsive positive, Eq. 26 without damping), delta_C, and the contact
 * radius a with x = a / a0.  Without adhesion (gamma == 0) JKR reduces to
 * Hertz: F = (4/3) E sqrt(R) delta^{3/2} and a = sqrt(R delta) for
 * delta >= 0, nothing below, delta_C = 0 and x = 0. */
static void normal_contact(double R, double E, double gamma, double delta, double* force,
                           double* dC, double* a, double* x) {
  if (gamma == 0.0) {
    double d = delta > 0.0 ? delta : 0.0;
    *force = 4.0 / 3.0 * E * sqrt(R) * d * sqrt(d);
    *dC = 0.0;
    *a = sqrt(R * d);
    *x = 0.0;
    return;
  }
  jkr_consts k = jkr_make(R, E, gamma);
  double xx = or_jkr_x(delta / k.dC);
  *force = 4.0 * k.FC * (xx * xx * xx - pow(xx, 1.5));
  *dC = k.dC;
  *a = xx * k.a0;
  *x = xx;
}

/* Elastic normal force and delta_C of a contact (normal_contact). */
void or_jkr_force(double R, double E, double gamma, double delta,
                  double* force, double* dC) {
  double a, x;
  normal_contact(R, E, gamma, delta, force, dC, &a, &x);
}

/* Position of id in a contact list of n entries, or -1. */
static int list_index(const int* ids, int n, int id) {
  for (int k = 0; k < n; ++k) if (ids[k] == id) return k;
  return -1;
}

static int in_list(const int* ids, int n, int id) { return list_index(ids, n, id) >= 0; }

/* The springs (xi[3], theta, xr[3], unused) that contact id carried in the
 * previous list (ids[n], springs hs[8n]), or zero for a new contact. */
static void prev_springs(const int* ids, int n, const double* hs, int id, double h[8]) {
  int k = list_index(ids, n, id);
  for (int b = 0; b < 8; ++b) h[b] = (k >= 0 && hs) ? hs[8 * k + b] : 0.0;
}

/* Velocity and spin of a body as friction sees them: a 2D disk moves in
 * its plane and spins about z only. */
static void planar(int two_d, const double* u, const double* w, double uo[3], double wo[3]) {
  for (int b = 0; b < 3; ++b) {
    uo[b] = u[b];
    wo[b] = w[b];
  }
  if (two_d) {
    uo[2] = 0.0;
    wo[0] = wo[1] = 0.0;
  }
}

static void cross(const double a[3], const double b[3], double out[3]) {
  out[0] = a[1] * b[2] - a[2] * b[1];
  out[1] = a[2] * b[0] - a[0] * b[2];
  out[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Sliding (Eq. 28 first line, cap Eq. 29 first line) and twisting (second
 * lines) of one contact; arguments as contact_friction, h[0..3]. */
static void sliding_twisting(const or_dem_params* p, const double n[3], double ri,
                             const double ui[3], const double wi[3], double rj,
                             const double uj[3], const double wj[3], double Fne, double FC,
                             double a, double dts, double h[4], double fc[3], double tc[3]) {
  double rin[3], rjn[3], si[3], sj[3], vR[3], vt[3];
  for (int b = 0; b < 3; ++b) {
    rin[b] = ri * n[b];
    rjn[b] = -rj * n[b];
  }
  cross(wi, rin, si);
  cross(wj, rjn, sj);
  for (int b = 0; b < 3; ++b) vR[b] = (uj[b] + sj[b]) - (ui[b] + si[b]);
  const double vn = dot3(vR, n);
  for (int b = 0; b < 3; ++b) vt[b] = vR[b] - vn * n[b];
  /* sliding (Eq. 28 first line, cap Eq. 29 first line) */
  const double Fcrit = p->mu_f * fabs(Fne + 2.0 * FC);
  const double hn = dot3(h, n);
  double xi[3], Ft[3];
  for (int b = 0; b < 3; ++b) {
    xi[b] = h[b] - hn * n[b] + dts * vt[b];
    Ft[b] = p->k_t * xi[b] + p->eta_t * vt[b];
  }
  const double Fmag = sqrt(dot3(Ft, Ft));
  if (Fmag > Fcrit) {
    for (int b = 0; b < 3; ++b) {
      Ft[b] *= Fcrit / Fmag;
      xi[b] = (Ft[b] - p->eta_t * vt[b]) / p->k_t;
    }
  }
  double tq[3];
  cross(rin, Ft, tq);
  for (int b = 0; b < 3; ++b) {
    fc[b] += Ft[b];
    tc[b] += tq[b];
    h[b] = xi[b];
  }
  /* twisting (Eq. 28 second line, cap Eq. 29 second line) */
  const double Om = dot3(wj, n) - dot3(wi, n);
  const double kr = 0.5 * p->k_t * a * a, er = 0.5 * p->eta_t * a * a;
  double theta = h[3] + dts * Om;
  double Mt = kr * theta + er * Om;
  const double Mcrit = 3.0 * M_PI * a * Fcrit / 16.0;
  if (fabs(Mt) > Mcrit) {
    Mt = Mt > 0.0 ? Mcrit : -Mcrit;
    theta = (Mt - er * Om) / kr;
  }
  for (int b = 0; b < 3; ++b) tc[b] += Mt * n[b];
  h[3] = theta;
}

/* Rolling resistance (Eq. 28 third line, cap Eq. 29 third line) of one
 * contact: the rolling displacement xr = integral of v_L with
 * v_L = R (w_i - w_j) x n, turned into the current tangent plane before the
 * sub-step's increment, resisted by the moment k_r |xr| with
 * k_r = 4 F_C x^{3/2}, which acts on i as k_r (xr x n).  Reading: Eq. 29's
 * M_r,crit is k_r theta_crit R in magnitude (its minus sign only restates
 * that the moment opposes the rolling), so the spring holds at most
 * |xr| = theta_crit R and is clamped there while the contact rolls on. */
static void rolling(const or_dem_params* p, const double n[3], double R, const double wi[3],
                    const double wj[3], double FC, double x, double dts, double xr[3],
                    double tc[3]) {
  double dw[3], dwn[3], m[3];
  for (int b = 0; b < 3; ++b) dw[b] = wi[b] - wj[b];
  cross(dw, n, dwn);                              /* v_L = R dwn */
  const double hn = dot3(xr, n);
  for (int b = 0; b < 3; ++b) xr[b] = xr[b] - hn * n[b] + dts * R * dwn[b];
  const double mag = sqrt(dot3(xr, xr)), cap = p->theta_r * R;
  if (mag > cap)
    for (int b = 0; b < 3; ++b) xr[b] *= cap / mag;
  const double kr = 4.0 * FC * pow(x, 1.5);
  cross(xr, n, m);
  for (int b = 0; b < 3; ++b) tc[b] += kr * m[b];
}

/* Sliding, twisting and rolling friction of one contact (Eqs. 22, 28, 29),
 * each a linear spring-dashpot-slider.  Body i (radius ri, velocity ui, spin
 * wi) touches body j (rj, uj, wj; a wall has zero velocity and spin) along
 * the unit normal n from i towards j; R is the effective radius.  Fne is the
 * elastic normal force (repulsive positive, no damping), FC = 3 pi gamma R,
 * a the contact radius and x = a / a0.  h holds the contact's springs from
 * the previous sub-step (the tangential displacement xi[3], the twist angle
 * theta and the rolling displacement xr[3]) and receives the new ones; the
 * force on i is added to fc and its torque about i's centre to tc.  Sliding
 * and twisting act with mu_f > 0, rolling with theta_r > 0 and adhesion.
 * Readings: v_R is the velocity of j's surface point relative to i's at the
 *   contact (points at distance ri and rj from the centres along n), and a
 *   positive displacement of j drags i along with it, which is the paper's
 *   minus sign with the roles of i and j exchanged; the integral of Eq. 28
 *   runs from the first sub-step of contact and includes the current one,
 *   and the stored displacement is projected onto the current tangent plane
 *   before the step's increment is added; min[.] caps the magnitude of the
 *   spring-plus-dashpot force (moment), and while it is capped the spring is
 *   reset to the stretch that gives the capped value (the slider takes the
 *   rest); F_ne of Eq. 29 is the elastic JKR force, so the cap
 *   mu_f (F_ne + 2 F_C) is positive on the whole stable branch. */
static void contact_friction(const or_dem_params* p, const double n[3], double ri,
                             const double ui[3], const double wi[3], double rj,
                             const double uj[3], const double wj[3], double R, double Fne,
                             double FC, double a, double x, double dts, double h[8],
                             double fc[3], double tc[3]) {
  if (p->mu_f > 0.0) sliding_twisting(p, n, ri, ui, wi, rj, uj, wj, Fne, FC, a, dts, h, fc, tc);
  if (p->theta_r > 0.0 && FC > 0.0) rolling(p, n, R, wi, wj, FC, x, dts, &h[4], tc);
}

/* One coupling step of the DEM (Eq. 21): n_sub semi-implicit Euler sub-steps
 * of dt / n_sub, with the hydrodynamic force Ff and torque Tf frozen (Sec.
 * 2.5).  Contacts (all pairs, nearest image) carry the JKR normal force with
 * the jump-on / pull-off hysteresis: a pair is in contact when its overlap is
 * >= 0, or when it is above -delta_C and the pair was in contact at the end
 * of the previous sub-step.  Reading: non-periodic axes have flat walls at
 * -1/2 and L-1/2 acting as JKR bodies of infinite radius and the particle's
 * material; the walls are contact partners -1-face.
 * gamma == 0 is Hertz's contact without adhesion (normal_contact).  With
 * mu_f > 0 or theta_r > 0 every contact also carries the friction of Eqs. 22,
 * 28, 29 (contact_friction); a wall is at rest.
 * Contact state: ncontact[np], contact_ids[np*cap] (sorted ascending), in/out;
 * hist[np*cap*8] (may be NULL without friction) holds each contact's springs
 * (xi[3], theta, xr[3], unused) beside its id; without friction the springs
 * are written as zero, so friction switched on later starts every persisting
 * contact unloaded.
 * Gravity G = (rho_p - rho_f) V g.  2D: disks of unit depth, V = pi r^2,
 * I = m r^2 / 2, spin about z only; 3D: V = 4/3 pi r^3, I = 2 m r^2 / 5.
 * Returns 0, or -1 when a particle has more than cap contacts. */
int or_dem_step(const or_config* c, const or_dem_params* p, int np, double* X,
                double* U, double* W, const double* R, const double* Ff,
                const double* Tf, int cap, int* ncontact, int* contact_ids, double* hist) {
  const int two_d = (c->q == 9);
  const double dts = p->dt / (double)p->n_sub;
  const int fric = p->mu_f > 0.0 || p->theta_r > 0.0;
  if (p->kinematic) {
    for (int sub = 0; sub < p->n_sub; ++sub)
      for (int s = 0; s < np; ++s)
        for (int a = 0; a < 3; ++a) X[3 * s + a] += dts * U[3 * s + a];
  } else {
    const double E = eff_modulus(p);
    double* Fc = (double*)calloc((size_t)3 * np, sizeof(double));
    double* Tc = (double*)calloc((size_t)3 * np, sizeof(double));
    int* nn = (int*)calloc((size_t)np, sizeof(int));
    int* nid = (int*)calloc((size_t)np * cap, sizeof(int));
    double* nh = (double*)calloc((size_t)np * cap * 8, sizeof(double));
    const double zero[3] = {0, 0, 0};
    int rc = 0;
    for (int sub = 0; sub < p->n_sub && rc == 0; ++sub) {
      for (int i = 0; i < np; ++i) {
        double fc[3] = {0, 0, 0}, tc[3] = {0, 0, 0};
        double hl[512][8];
        int cnt = 0, list[512];
        const int* prev = &contact_ids[(size_t)i * cap];
        const double* prev_h = hist ? &hist[(size_t)i * cap * 8] : NULL;
        /* particle-wall contacts first (ids -1-face are the smallest) */
        for (int face = 5; face >= 0; --face) {
          int a = face / 2;
          if (axis_periodic(c, a)) continue;
          double L = (double)dims(c, a);
          double dist = (face % 2 == 0) ? X[3 * i + a] + 0.5 : (L - 0.5) - X[3 * i + a];
          double delta = R[i] - dist, force, dC, acon, xcon;
          normal_contact(R[i], E, p->gamma, delta, &force, &dC, &acon, &xcon);
          int id = -1 - face;
          if (delta >= 0.0 || (delta > -dC && in_list(prev, ncontact[i], id))) {
            double nrm[3] = {0, 0, 0}, h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            nrm[a] = (face % 2 == 0) ? -1.0 : 1.0;
            double vrn = -(U[3 * i + 0] * nrm[0] + U[3 * i + 1] * nrm[1] + U[3 * i + 2] * nrm[2]);
            for (int b = 0; b < 3; ++b) fc[b] += (-force + p->eta_n * vrn) * nrm[b];
            if (fric) {
              double ui[3], wi[3];
              planar(two_d, &U[3 * i], &W[3 * i], ui, wi);
              prev_springs(prev, ncontact[i], prev_h, id, h);
              contact_friction(p, nrm, R[i], ui, wi, 0.0, zero, zero, R[i], force,
                               3.0 * M_PI * p->gamma * R[i], acon, xcon, dts, h, fc, tc);
            }
            if (cnt < 512) {
              list[cnt] = id;
              for (int b = 0; b < 8; ++b) hl[cnt][b] = h[b];
            }
            ++cnt;
          }
        }
        for (int j = 0; j < np; ++j) {
          if (j == i) continue;
          double dv[3], d2 = 0.0;
          for (int a = 0; a < 3; ++a) {
            if (a == 2 && two_d) { dv[a] = 0.0; continue; }
            dv[a] = min_image(c, a, X[3 * j + a] - X[3 * i + a]);
            d2 += dv[a] * dv[a];
          }
          double dist = sqrt(d2);
          double delta = R[i] + R[j] - dist;
          double Reff = 1.0 / (1.0 / R[i] + 1.0 / R[j]);
          if (delta < 0.0 && !in_list(prev, ncontact[i], j)) continue;
          double force, dC, acon, xcon;
          normal_contact(Reff, E, p->gamma, delta, &force, &dC, &acon, &xcon);
          if (delta >= 0.0 || delta > -dC) {
            double nrm[3], vrn = 0.0, h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int a = 0; a < 3; ++a) nrm[a] = dv[a] / dist;
            for (int a = 0; a < 3; ++a) vrn += (U[3 * j + a] - U[3 * i + a]) * nrm[a];
            for (int a = 0; a < 3; ++a) fc[a] += (-force + p->eta_n * vrn) * nrm[a];
            if (fric) {
              double ui[3], wi[3], uj[3], wj[3];
              planar(two_d, &U[3 * i], &W[3 * i], ui, wi);
              planar(two_d, &U[3 * j], &W[3 * j], uj, wj);
              prev_springs(prev, ncontact[i], prev_h, j, h);
              contact_friction(p, nrm, R[i], ui, wi, R[j], uj, wj, Reff, force,
                               3.0 * M_PI * p->gamma * Reff, acon, xcon, dts, h, fc, tc);
            }
            if (cnt < 512) {
              list[cnt] = j;
              for (int b = 0; b < 8; ++b) hl[cnt][b] = h[b];
            }
            ++cnt;
          }
        }
        if (cnt > cap) { rc = -1; break; }
        nn[i] = cnt;
        for (int k = 0; k < cnt; ++k) {
          nid[(size_t)i * cap + k] = list[k];
          for (int b = 0; b < 8; ++b) nh[((size_t)i * cap + k) * 8 + b] = hl[k][b];
        }
        for (int a = 0; a < 3; ++a) {
          Fc[3 * i + a] = fc[a];
          Tc[3 * i + a] = tc[a];
        }
      }
      if (rc) break;
      for (int i = 0; i < np; ++i) {
        double r = R[i];
        double V = two_d ? M_PI * r * r : (4.0 / 3.0) * M_PI * r * r * r;
        double m = p->rho_p * V;
        double I = two_d ? 0.5 * m * r * r : 0.4 * m * r * r;
        for (int a = 0; a < 3; ++a) {
          if (a == 2 && two_d) continue;
          double G = (p->rho_p - p->rho_f) * V * p->g[a];
          U[3 * i + a] += dts * (Ff[3 * i + a] + Fc[3 * i + a] + G) / m;
          X[3 * i + a] += dts * U[3 * i + a];
        }
        if (two_d) {
          W[3 * i + 2] += dts * (Tf[3 * i + 2] + Tc[3 * i + 2]) / I;
        } else {
          for (int a = 0; a < 3; ++a) W[3 * i + a] += dts * (Tf[3 * i + a] + Tc[3 * i + a]) / I;
        }
        ncontact[i] = nn[i];
        for (int k = 0; k < nn[i]; ++k) {
          contact_ids[(size_t)i * cap + k] = nid[(size_t)i * cap + k];
          if (hist)
            for (int b = 0; b < 8; ++b)
              hist[((size_t)i * cap + k) * 8 + b] = nh[((size_t)i * cap + k) * 8 + b];
        }
      }
    }
    free(Fc); free(Tc); free(nn); free(nid); free(nh);
    if (rc) return rc;
  }
  /* wrap positions into [0, L) on periodic axes */
  for (int s = 0; s < np; ++s)
    for (int a = 0; a < 3; ++a) {
      if (a == 2 && two_d) continue;
      if (!axis_periodic(c, a)) continue;
      double L = (double)dims(c, a);
      if (X[3 * s + a] >= L) X[3 * s + a] -= L;
      else if (X[3 * s + a] < 0.0) X[3 * s + a] += L;
    }
  return 0;
}
