// Adhesive DEM step of the gfx950 PSC-LBM library (FP64), Sec. 2.5:
// Newton-Euler motion (Eq. 21) with the JKR normal contact force (Eqs. 25-27)
// including the jump-on / pull-off hysteresis and, optionally, the sliding
// and twisting friction of Eqs. 22, 28, 29, sub-cycled n_sub times per
// coupling step with the hydrodynamic force and torque held fixed.
//
// Per sub-step, two kernels: (1) bin the particles into a uniform grid whose
// bins are at least 2 r_max + 1 wide, each bin entry a record of the
// particle's position, velocity, radius and id; (2) one wave per particle
// gathers its contacts from the records of the neighbouring bins and the
// walls (so that no particle sees another's update), records the new contact
// list, sums the forces over the wave and integrates the particle with
// semi-implicit Euler.  The bin counts and records are triple buffered: each
// binning fills one set and clears the set the binning after it fills.  With
// friction the binning also copies the spins, which the contacts read, and
// each contact's springs travel with the contact lists.
//
// The coupled step (n_sub = 1) gathers the contacts in leading workgroups of
// the step kernel instead, which run beside the tiles (contacts need only
// the binning of the step's start); its DEM kernel reads their forces,
// integrates, and rasterises and bins the particles for the next step.  With
// friction or the Hertz contact the DEM kernel gathers the contacts itself
// from that binning, and records the spins for the next step's contacts.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "common.hpp"
#include "dem.hpp"
#include "tiles.hpp"

namespace psclbm {


// One thread per particle: its bin in the target set and its image; the
// grid also clears the set the binning after next fills.  wsnap (friction
// only): a copy of the spins at the start of the sub-step.
__global__ void k_dem_bin(DemBinOut b, Geom g, int n, int three_d, const double* x,
                          const double* u, const double* r, unsigned* err, const double* w,
                          double* wsnap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  for (long long k = i; k < b.nbins; k += (long long)gridDim.x * blockDim.x) b.stale[k] = 0;
  if (i >= n) return;
  dem_bin_insert(b, three_d, g, i, x + 3 * i, u + 3 * i, r[i], err);
  if (wsnap)
    for (int a = 0; a < 3; ++a) wsnap[3 * i + a] = w[3 * i + a];
}

struct IntArgs {
  int n, three_d;
  int L[3], periodic[3];
  double dt;
  double rho_p, rho_f;
  double g[3];
  int kinematic;
  int wrap;
  int fstride, tstride;  // element strides of the force / torque rows
};

// Semi-implicit Euler (Eq. 21) with hydrodynamic force F, torque T, contact
// force fc and contact torque tc (null: none): u += dt (F + fc + G)/m,
// x += dt u, omega += dt (T + tc)/I, then the wrap into [0, L) on periodic
// axes (kinematic: x += dt u only).
__device__ inline void integrate_state(const IntArgs& p, double ri, const double* F,
                                       const double* T, const double* fc, const double* tc,
                                       double* x, double* u, double* w) {
  const int D = p.three_d ? 3 : 2;
  if (!p.kinematic) {
    const double V = p.three_d ? (4.0 / 3.0) * M_PI * ri * ri * ri : M_PI * ri * ri;
    const double m = p.rho_p * V;
    const double I = p.three_d ? 0.4 * m * ri * ri : 0.5 * m * ri * ri;
    for (int a = 0; a < D; ++a) {
      const double G = (p.rho_p - p.rho_f) * V * p.g[a];
      u[a] += p.dt * (F[a] + fc[a] + G) / m;
      x[a] += p.dt * u[a];
    }
    if (p.three_d) {
      for (int a = 0; a < 3; ++a) w[a] += p.dt * (tc ? T[a] + tc[a] : T[a]) / I;
    } else {
      w[2] += p.dt * (tc ? T[2] + tc[2] : T[2]) / I;
    }
  } else {
    for (int a = 0; a < D; ++a) x[a] += p.dt * u[a];
  }
  if (p.wrap) {
    for (int a = 0; a < D; ++a) {
      if (!p.periodic[a]) continue;
      const double L = (double)p.L[a];
      if (x[a] >= L) x[a] -= L;
      else if (x[a] < 0.0) x[a] += L;
    }
  }
}

// Rasterisation of the next coupled step by the DEM wave of this one: the
// tile set to fill (all zero on entry) and the one to clear, the snapshot and
// the DEM binning of the updated particle.
struct NextOut {
  int build;
  Geom g;
  double h;
  PSnap* snap;
  int* tcount;
  int* tstale;
  long long ntiles;
  int* tile_list;
  int cap;
  DemBinOut db;
  double* wnext;  // friction: the updated spins, which the next step's contacts read
  unsigned* err;
};

// One wave per particle.  Unless fc_in holds them (the contact forces the
// coupled step kernel gathered), the contacts are gathered here
// (dem_contact_wave, with friction when FRIC and Hertz's normal force when
// HERTZ).  Every lane then integrates the particle (the same values), lane 0
// stores it, and with nx.build the wave rasterises it for the next coupled
// step.  Kinematic particles skip the contacts.
template <bool FRIC, bool HERTZ>
__global__ void __launch_bounds__(256) k_dem_contacts(DemArgs d, FricArgs fr, IntArgs ia,
                                                      NextOut nx, double* x, double* u,
                                                      double* w, const double* r,
                                                      const double* Ff, const double* Tf,
                                                      const double* fc_in) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (nx.build) {
    for (long long k = gid; k < nx.ntiles; k += (long long)gridDim.x * blockDim.x)
      nx.tstale[k] = 0;
    if (nx.db.count)
      for (long long k = gid; k < nx.db.nbins; k += (long long)gridDim.x * blockDim.x)
        nx.db.stale[k] = 0;
  }
  const int i = (int)(gid >> 6);
  const int lane = (int)(threadIdx.x & 63);
  if (i >= d.n) return;  // uniform over the wave
  const int D = d.three_d ? 3 : 2;
  const double ri = r[i];
  // the particle's previous snapshot: its c_s is reused while r is unchanged
  double r_prev = -1.0, cs_prev = 0.0;
  if (nx.build) {
    r_prev = nx.snap[i].r;
    cs_prev = nx.snap[i].cs;
  }
  double xs[3], us[3], ws[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    xs[a] = x[3 * i + a];
    us[a] = u[3 * i + a];
    ws[a] = w[3 * i + a];
  }
  double fsum[3] = {0.0, 0.0, 0.0};
  double tsum[3] = {0.0, 0.0, 0.0};
  if constexpr (FRIC || HERTZ) {
    dem_contact_wave<FRIC, HERTZ>(d, i, lane, xs, us, ri, fsum, &fr, ws, tsum);
  } else if (fc_in) {  // contacts gathered by the step kernel's contact workgroups
#pragma unroll
    for (int a = 0; a < 3; ++a) fsum[a] = fc_in[3 * i + a];
  } else if (!ia.kinematic) {
    dem_contact_wave(d, i, lane, xs, us, ri, fsum);
  }
  integrate_state(ia, ri, Ff + (size_t)ia.fstride * i, Tf + (size_t)ia.tstride * i, fsum,
                  FRIC ? tsum : nullptr, xs, us, ws);
  if (lane == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      x[3 * i + a] = xs[a];
      u[3 * i + a] = us[a];
      w[3 * i + a] = ws[a];
    }
  }
  if (!nx.build) return;
  PSnap P;
  const bool ok = make_snap(d.three_d, xs, us, ws, ri, P, r_prev, cs_prev);
  if (lane == 0) {
    nx.snap[i] = P;
    if (!ok) atomicOr(nx.err, ERR_RADIUS);
    if (nx.db.count) dem_bin_insert(nx.db, d.three_d, nx.g, i, xs, us, ri, nx.err);
    if constexpr (FRIC) {
      if (nx.wnext)
        for (int a = 0; a < 3; ++a) nx.wnext[3 * i + a] = ws[a];
    }
  }
  if (ok) bin_tiles(nx.g, d.three_d, nx.h, P, i, lane, nx.tcount, nx.tile_list, nx.cap, nx.err);
}

// Kinematic particles (prescribed velocities): x += dt u.
__global__ void k_dem_advect(IntArgs p, double* x, double* u, double* w, const double* r,
                             const double* Ff, const double* Tf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const double z[3] = {0.0, 0.0, 0.0};
  integrate_state(p, r[i], Ff + (size_t)p.fstride * i, Tf + (size_t)p.tstride * i, z, nullptr,
                  x + 3 * i, u + 3 * i, w + 3 * i);
}

int launch_dem_reset(psclbm_ctx* c) {
  if (c->cfg.max_particles <= 0) return PSCLBM_OK;
  return hip_ok(hipMemsetAsync(c->contact_n[c->contact_cur], 0,
                               sizeof(int) * (size_t)c->cfg.max_particles, c->stream));
}

static IntArgs int_args(const psclbm_ctx* c, const psclbm_dem_params* prm, int n,
                        const double*& F, const double*& T) {
  IntArgs ia;
  ia.n = n;
  ia.three_d = c->geom.q == 19;
  ia.L[0] = c->geom.nx;
  ia.L[1] = c->geom.ny;
  ia.L[2] = c->geom.nz;
  for (int a = 0; a < 3; ++a) {
    ia.periodic[a] = c->geom.periodic[a];
    ia.g[a] = prm->g[a];
  }
  ia.dt = prm->dt / prm->n_sub;
  ia.rho_p = prm->rho_p;
  ia.rho_f = prm->rho_f;
  ia.kinematic = prm->kinematic ? 1 : 0;
  ia.wrap = 1;
  // NULL force and torque: the FP64 accumulators of the most recent lbm_step
  ia.fstride = 3;
  ia.tstride = 3;
  if (!F && !T) {
    F = c->facc[c->force_buf];
    T = F + 3;
    ia.fstride = ia.tstride = 6;
  }
  return ia;
}

// Effective modulus of two bodies of the material (Eq. 25); 0 when the
// contact reach delta_C of the largest pair does not fit in the bin margin.
static double dem_modulus(const psclbm_ctx* c, const psclbm_dem_params* prm) {
  const double E = 1.0 / (2.0 * (1.0 - prm->poisson * prm->poisson) / prm->E_p);
  const double Rm = c->cfg.max_radius;  // wall contact: R = r
  const double a0 = std::cbrt(9.0 * M_PI * prm->gamma * Rm * Rm / E);
  const double dC = a0 * a0 / (2.0 * std::cbrt(6.0) * Rm);
  return dC < 1.0 ? E : 0.0;
}

// Contact-pass arguments on the current binning and contact lists.
static DemArgs dem_args(const psclbm_ctx* c, const psclbm_dem_params* prm, int n, double E) {
  DemArgs d;
  d.n = n;
  d.three_d = c->geom.q == 19;
  d.L[0] = c->geom.nx;
  d.L[1] = c->geom.ny;
  d.L[2] = c->geom.nz;
  for (int a = 0; a < 3; ++a) {
    d.periodic[a] = c->geom.periodic[a];
    d.nbin[a] = c->nbin[a];
    d.bin_size[a] = c->bin_size[a];
  }
  d.bin_cap = c->bin_cap;
  d.bin_count = c->bin_count_buf[c->bin_cur];
  d.bin_rec = c->bin_rec[c->bin_cur];
  d.prev_n = c->contact_n[c->contact_cur];
  d.prev_id = c->contact_id[c->contact_cur];
  d.next_n = c->contact_n[c->contact_cur ^ 1];
  d.next_id = c->contact_id[c->contact_cur ^ 1];
  d.max_contacts = c->cfg.max_contacts;
  d.E = E;
  d.gamma = prm->gamma;
  d.eta_n = prm->eta_n;
  d.err = c->err;
  return d;
}

// Friction of any kind is on: the contacts keep springs.
static bool dem_friction(const psclbm_dem_params* prm) {
  return prm->mu_f > 0.0 || prm->theta_r > 0.0;
}

// Friction arguments of a contact pass that reads the spins wsnap: the
// springs of the current lists (if they were kept) and those being built.
static FricArgs fric_args(psclbm_ctx* c, const psclbm_dem_params* prm, const double* wsnap) {
  FricArgs fr;
  std::memset(&fr, 0, sizeof(fr));
  fr.w = wsnap;
  fr.prev_h = c->springs_valid ? c->contact_springs[c->contact_cur] : nullptr;
  fr.next_h = c->contact_springs[c->contact_cur ^ 1];
  fr.k_t = prm->k_t;
  fr.eta_t = prm->eta_t;
  fr.mu_f = prm->mu_f;
  fr.theta_r = prm->theta_r;
  fr.dts = prm->dt / prm->n_sub;
  return fr;
}

// k_dem_contacts in the instantiation for friction and the Hertz contact.
static int launch_contacts(psclbm_ctx* c, bool fric, bool hertz, int n, const DemArgs& d,
                           const FricArgs& fr, const IntArgs& ia, const NextOut& nx, double* x,
                           double* u, double* w, const double* r, const double* F,
                           const double* T, const double* fc_in) {
  const dim3 grid((n + 3) / 4), block(256);
  if (fric && hertz)
    k_dem_contacts<true, true><<<grid, block, 0, c->stream>>>(d, fr, ia, nx, x, u, w, r, F, T,
                                                             fc_in);
  else if (fric)
    k_dem_contacts<true, false><<<grid, block, 0, c->stream>>>(d, fr, ia, nx, x, u, w, r, F, T,
                                                              fc_in);
  else if (hertz)
    k_dem_contacts<false, true><<<grid, block, 0, c->stream>>>(d, fr, ia, nx, x, u, w, r, F, T,
                                                              fc_in);
  else
    k_dem_contacts<false, false><<<grid, block, 0, c->stream>>>(d, fr, ia, nx, x, u, w, r, F,
                                                               T, fc_in);
  return hip_ok(hipGetLastError());
}

int launch_dem_step(psclbm_ctx* c, const psclbm_dem_params* prm, double* x, double* u, double* w,
                    const double* r, int n, const double* F, const double* T) {
  IntArgs ia = int_args(c, prm, n, F, T);
  const int blocks = (n + 127) / 128;
  if (prm->kinematic) {
    for (int s = 0; s < prm->n_sub; ++s) {
      ia.wrap = s == prm->n_sub - 1;
      k_dem_advect<<<blocks, 128, 0, c->stream>>>(ia, x, u, w, r, F, T);
      int rc = hip_ok(hipGetLastError());
      if (rc) return rc;
    }
    return PSCLBM_OK;
  }
  const double E = dem_modulus(c, prm);
  if (!(E > 0.0)) return PSCLBM_EINVAL;
  NextOut nx;
  std::memset(&nx, 0, sizeof(nx));
  const bool fric = dem_friction(prm), hertz = prm->gamma == 0.0;
  for (int s = 0; s < prm->n_sub; ++s) {
    ia.wrap = s == prm->n_sub - 1;  // positions wrap once, after the last sub-step
    const DemBinOut b = dem_bin_out(c, true);
    const long long bth = b.nbins > n ? b.nbins : n;
    k_dem_bin<<<(unsigned)((bth + 127) / 128), 128, 0, c->stream>>>(
        b, c->geom, n, c->geom.q == 19, x, u, r, c->err, w, fric ? c->wsnap[0] : nullptr);
    dem_bins_advance(c);
    const DemArgs d = dem_args(c, prm, n, E);
    const FricArgs fr = fric_args(c, prm, c->wsnap[0]);
    const int rc = launch_contacts(c, fric, hertz, n, d, fr, ia, nx, x, u, w, r, F, T, nullptr);
    if (rc) return rc;
    c->contact_cur ^= 1;
    c->springs_valid = fric ? 1 : 0;
  }
  return PSCLBM_OK;
}

int launch_coupled(psclbm_ctx* c, const psclbm_dem_params* prm, double* x, double* u, double* w,
                   const double* r, int n, int nsteps) {
  psclbm_particles pp;
  pp.n = n;
  pp.x = x;
  pp.u = u;
  pp.omega = w;
  pp.radius = r;
  const psclbm_particles* p = &pp;
  double E = 0.0;
  if (!prm->kinematic) {
    E = dem_modulus(c, prm);
    if (!(E > 0.0)) return PSCLBM_EINVAL;
  }
  if (prm->n_sub != 1 || n == 0) {
    // sub-cycled DEM: the three calls in turn
    for (int t = 0; t < nsteps; ++t) {
      int rc = launch_rasterize(c, p, false);
      if (!rc) c->np = n;
      if (!rc) rc = launch_step(c);
      if (!rc && n > 0)
        rc = launch_dem_step(c, prm, x, u, w, r, n, nullptr, nullptr);
      if (rc) return rc;
    }
    return PSCLBM_OK;
  }
  // with friction or the Hertz contact the DEM kernel gathers the contacts
  const bool fric = !prm->kinematic && dem_friction(prm);
  const bool hertz = !prm->kinematic && prm->gamma == 0.0;
  const bool own_contacts = prm->kinematic || fric || hertz;
  // first step's rasterisation, with its DEM binning (and spins)
  int rc = launch_rasterize(c, p, !prm->kinematic);
  if (!rc && fric)
    rc = hip_ok(hipMemcpyAsync(c->wsnap[0], w, sizeof(double) * 3 * (size_t)n,
                               hipMemcpyDeviceToDevice, c->stream));
  if (rc) return rc;
  c->np = n;
  const size_t ntiles = (size_t)c->ntiles;
  int wcur = 0;  // the spin snapshot of the current step's start
  for (int t = 0; t < nsteps; ++t) {
    // the step, with the contact workgroups on the binning of its start
    const DemArgs d = dem_args(c, prm, n, E);
    rc = own_contacts ? launch_step(c) : launch_step_contacts(c, &d, x, u, r);
    if (rc) return rc;
    const bool build = t + 1 < nsteps;
    const double* F = nullptr;
    const double* T = nullptr;
    const IntArgs ia = int_args(c, prm, n, F, T);
    NextOut nx;
    std::memset(&nx, 0, sizeof(nx));
    nx.build = build ? 1 : 0;
    nx.g = c->geom;
    nx.h = c->cfg.shell_h;
    nx.snap = c->snap;
    nx.tcount = c->tile_count_buf[c->tile_cur ^ 1];
    nx.tstale = c->tile_count_buf[c->tile_cur];
    nx.ntiles = (long long)ntiles;
    nx.tile_list = c->tile_list;
    nx.cap = c->cfg.max_tile_particles;
    nx.db = dem_bin_out(c, build && !prm->kinematic);
    nx.wnext = build && fric ? c->wsnap[wcur ^ 1] : nullptr;
    nx.err = c->err;
    const FricArgs fr = fric_args(c, prm, c->wsnap[wcur]);
    rc = launch_contacts(c, fric, hertz, n, d, fr, ia, nx, x, u, w, r, F, T,
                         own_contacts ? nullptr : c->fcontact);
    if (rc) return rc;
    if (!prm->kinematic) {
      c->contact_cur ^= 1;
      c->springs_valid = fric ? 1 : 0;
    }
    wcur ^= 1;
    if (build) {
      c->tile_cur ^= 1;
      c->tile_count = c->tile_count_buf[c->tile_cur];
      if (nx.db.count) dem_bins_advance(c);
    }
  }
  return PSCLBM_OK;
}


// ------------------------------------------------------------------------
// Adjoint of one frictionless DEM step (n_sub = 1) with its contact set held
// fixed (the jump-on / pull-off switches contribute nothing).  With
// s_i = dt/m_i (du'_i + dt dx'_i), the adjoint of the contact force of i, and
// the pair force g_ij = (-F(delta) + eta_n (u_j - u_i).n) n = -g_ji:
//   dx_i = dx'_i + sum_j (d g_ij / d x_i)^T (s_i - s_j),
//   du_i = du'_i + dt dx'_i + sum_j (d g_ij / d u_i)^T (s_i - s_j),
// where walls take s_j = 0; dF = s, dT = dt/I dw', dw = dw'.
// ------------------------------------------------------------------------

// dF/d delta of the elastic normal force at overlap delta (x = a/a0 from the
// force evaluation).  JKR: F = 4 F_C (x^3 - x^{3/2}) and
// delta = delta_C 6^{1/3} (2 x^2 - 4/3 x^{1/2}), so the slope is the ratio
// of their x-derivatives; zero where the branch is clamped at pull-off.
// Hertz (gamma = 0): (3/2) (4/3) E sqrt(R) delta^{1/2}.
__device__ inline double normal_slope(double R, double E, double gamma, double delta, double x) {
  if (gamma == 0.0) return delta > 0.0 ? 2.0 * E * sqrt(R) * sqrt(delta) : 0.0;
  const double c6 = 1.8171205928321397;  // 6^{1/3}
  const double FC = 3.0 * M_PI * gamma * R;
  const double a0 = cbrt(9.0 * M_PI * gamma * R * R / E);
  const double dc = a0 * a0 / (2.0 * c6 * R);
  const double sC = 1.0 / c6;
  if ((delta / dc) / c6 <= 2.0 * sC * sC * sC * sC - (4.0 / 3.0) * sC) return 0.0;
  const double sx = sqrt(x);
  return 4.0 * FC * (3.0 * x * x - 1.5 * sx) / (dc * c6 * (4.0 * x - (2.0 / 3.0) / sx));
}

// One thread per particle: s_i (written as dF), dT and dw.
__global__ void k_dem_adj_seed(IntArgs p, const double* r, const double* gx, const double* gu,
                               const double* gw, double* aF, double* aT, double* aw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const int D = p.three_d ? 3 : 2;
  const double ri = r[i];
  const double V = p.three_d ? (4.0 / 3.0) * M_PI * ri * ri * ri : M_PI * ri * ri;
  const double m = p.rho_p * V;
  const double I = p.three_d ? 0.4 * m * ri * ri : 0.5 * m * ri * ri;
  for (int a = 0; a < 3; ++a) {
    const double up = gu[3 * i + a] + (a < D ? p.dt * gx[3 * i + a] : 0.0);
    aF[3 * i + a] = a < D ? p.dt * up / m : 0.0;
    aT[3 * i + a] = (p.three_d || a == 2) ? p.dt * gw[3 * i + a] / I : 0.0;
    aw[3 * i + a] = gw[3 * i + a];
  }
}

// One wave per particle, one lane per contact of the step's list (at most 64).
__global__ void __launch_bounds__(256) k_dem_adj_gather(DemArgs d, IntArgs p, const double* x,
                                                        const double* u, const double* r,
                                                        const double* gx, const double* gu,
                                                        const double* s, double* ax,
                                                        double* au) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(gid >> 6);
  const int lane = (int)(threadIdx.x & 63);
  if (i >= d.n) return;  // uniform over the wave
  const int D = d.three_d ? 3 : 2;
  int cnt = d.prev_n[i];
  if (cnt > d.max_contacts) cnt = d.max_contacts;
  double bx[3] = {0.0, 0.0, 0.0}, bu[3] = {0.0, 0.0, 0.0};
  if (lane < cnt) {
    const int id = d.prev_id[(size_t)i * d.max_contacts + lane];
    const double ri = r[i];
    // (partners outside this call's particles or walls of other lattices,
    // as a list left by a larger step could hold, are skipped)
    if (id < 0 && -1 - id < 2 * D) {  // wall: n = sgn e_a, d delta / d x_a = sgn, s_j = 0
      const int face = -1 - id, a = face / 2;
      const double xa = x[3 * i + a];
      const double dist = (face % 2 == 0) ? xa + 0.5 : (d.L[a] - 0.5) - xa;
      const double delta = ri - dist;
      double dC, acon, xcon = 0.0;
      if (d.gamma == 0.0) hertz_force(ri, d.E, delta, &acon);
      else jkr_force(ri, d.E, d.gamma, delta, &dC, &acon, &xcon);
      const double Fp = normal_slope(ri, d.E, d.gamma, delta, xcon);
      const double v = s[3 * i + a];
      bx[a] = -Fp * v;
      bu[a] = -d.eta_n * v;
    } else if (id >= 0 && id < d.n) {
      const int j = id;
      double dv[3], du[3], v[3];
      for (int a = 0; a < 3; ++a) {
        const bool on = a < D;
        dv[a] = on ? min_img(x[3 * j + a] - x[3 * i + a], d.periodic[a], d.L[a]) : 0.0;
        du[a] = on ? u[3 * j + a] - u[3 * i + a] : 0.0;
        v[a] = on ? s[3 * i + a] - s[3 * j + a] : 0.0;
      }
      const double rho = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
      const double n0 = dv[0] / rho, n1 = dv[1] / rho, n2 = dv[2] / rho;
      const double rj = r[j];
      const double delta = ri + rj - rho;
      const double Reff = 1.0 / (1.0 / ri + 1.0 / rj);
      double dC, acon, xcon = 0.0, F;
      if (d.gamma == 0.0) F = hertz_force(Reff, d.E, delta, &acon);
      else F = jkr_force(Reff, d.E, d.gamma, delta, &dC, &acon, &xcon);
      const double Fp = normal_slope(Reff, d.E, d.gamma, delta, xcon);
      const double dun = du[0] * n0 + du[1] * n1 + du[2] * n2;
      const double phi = -F + d.eta_n * dun;
      const double vn = v[0] * n0 + v[1] * n1 + v[2] * n2;
      const double nn[3] = {n0, n1, n2};
      for (int a = 0; a < 3; ++a) {
        const double Pdu = du[a] - dun * nn[a], Pv = v[a] - vn * nn[a];
        bx[a] = (-Fp * nn[a] - d.eta_n * Pdu / rho) * vn - phi * Pv / rho;
        bu[a] = -d.eta_n * nn[a] * vn;
      }
    }
  }
  for (int a = 0; a < 3; ++a) {
    bx[a] = wave_sum(bx[a]);
    bu[a] = wave_sum(bu[a]);
  }
  if (lane == 0) {
    for (int a = 0; a < 3; ++a) {
      const double gxa = gx[3 * i + a];
      ax[3 * i + a] = gxa + bx[a];
      au[3 * i + a] = gu[3 * i + a] + (a < D ? p.dt * gxa : 0.0) + bu[a];
    }
  }
}

int launch_dem_adjoint(psclbm_ctx* c, const psclbm_dem_params* prm, const double* x,
                       const double* u, const double* r, int n, const double* gx,
                       const double* gu, const double* gw, double* ax, double* au, double* aw,
                       double* aF, double* aT) {
  const double E = dem_modulus(c, prm);
  if (!(E > 0.0)) return PSCLBM_EINVAL;
  const double* F = nullptr;
  const double* T = nullptr;
  const IntArgs ia = int_args(c, prm, n, F, T);
  // the contact lists of the step just taken are the current ones
  const DemArgs d = dem_args(c, prm, n, E);
  k_dem_adj_seed<<<(n + 127) / 128, 128, 0, c->stream>>>(ia, r, gx, gu, gw, aF, aT, aw);
  int rc = hip_ok(hipGetLastError());
  if (rc) return rc;
  k_dem_adj_gather<<<(n + 3) / 4, 256, 0, c->stream>>>(d, ia, x, u, r, gx, gu, aF, ax, au);
  return hip_ok(hipGetLastError());
}

}  // namespace psclbm
