// extern "C" entry points of the gfx950 PSC-LBM library (see include/psclbm.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "common.hpp"

namespace psclbm {
// Adjoint of the DEM step just taken (dem.hip).
int launch_dem_adjoint(psclbm_ctx* c, const psclbm_dem_params* prm, const double* x,
                       const double* u, const double* r, int n, const double* gx,
                       const double* gu, const double* gw, double* ax, double* au, double* aw,
                       double* aF, double* aT);
}  // namespace psclbm

using namespace psclbm;

namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

inline int storage_bytes(int prec) {
  return prec == PSCLBM_FP64 ? 8 : (prec == PSCLBM_FP32 ? 4 : 2);
}

bool axis_is_periodic(const psclbm_config* c, int a) {
  if (a == 2 && c->lattice == 9) return true;
  return c->face_bc[2 * a] == PSCLBM_PERIODIC;
}

// Validates a configuration; 0 when usable.
int validate(const psclbm_config* c) {
  if (!c) return PSCLBM_EINVAL;
  if (c->lattice != 9 && c->lattice != 19) return PSCLBM_EINVAL;
  if (c->nx < 1 || c->ny < 1 || c->nz < 1) return PSCLBM_EINVAL;
  if (c->lattice == 9 && c->nz != 1) return PSCLBM_EINVAL;
  if (!(c->tau > 0.5) || !std::isfinite(c->tau)) return PSCLBM_EINVAL;
  if (!(c->rho0 > 0.0) || !std::isfinite(c->rho0)) return PSCLBM_EINVAL;
  if (!(c->shell_h >= 0.0) || !std::isfinite(c->shell_h)) return PSCLBM_EINVAL;
  if (c->precision < PSCLBM_FP64 || c->precision > PSCLBM_FP32_FP16STORE) return PSCLBM_EINVAL;
  if (c->weighting != PSCLBM_WEIGHT_MODIFIED && c->weighting != PSCLBM_WEIGHT_ORIGINAL)
    return PSCLBM_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(c->body_force[k])) return PSCLBM_EINVAL;
  const int L[3] = {c->nx, c->ny, c->nz};
  for (int a = 0; a < (c->lattice == 9 ? 2 : 3); ++a) {
    const int f0 = c->face_bc[2 * a], f1 = c->face_bc[2 * a + 1];
    for (int f : {f0, f1})
      if (f < PSCLBM_PERIODIC || f > PSCLBM_OUTLET_EQ) return PSCLBM_EINVAL;
    if ((f0 == PSCLBM_PERIODIC) != (f1 == PSCLBM_PERIODIC)) return PSCLBM_EINVAL;
    for (int f : {f0, f1})
      if ((f == PSCLBM_INLET_EQ || f == PSCLBM_OUTLET_EQ) && L[a] < 3) return PSCLBM_EINVAL;
  }
  for (int f = 0; f < 6; ++f)
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(c->face_velocity[f][k])) return PSCLBM_EINVAL;
  if (c->max_particles < 0) return PSCLBM_EINVAL;
  if (c->max_particles > 0) {
    if (c->max_tile_particles < 1 || c->max_tile_particles > 512) return PSCLBM_EINVAL;
    if (c->max_contacts < 1 || c->max_contacts > 64) return PSCLBM_EINVAL;
    if (!(c->max_radius > 0.0) || !std::isfinite(c->max_radius)) return PSCLBM_EINVAL;
  }
  // the kernels address one direction's array with 32-bit byte offsets
  const double cells = (double)c->nx * c->ny * c->nz;
  if (cells * storage_bytes(c->precision) >= 4294967296.0) return PSCLBM_EINVAL;
  return PSCLBM_OK;
}

// Tile width along x.  3D: the widest of 256, 128 and 64 cells that pads the
// x extent least (a tile row is four, two or one 64-cell wave segments); wide
// tiles keep the cache lines that the odd steps' shifted accesses split
// between neighbouring segments inside one workgroup (256^3 FP32 odd step 483
// against 531-556 us with 64-wide tiles).  2D: 64 x 4 tiles, whose four rows
// share one short particle list (512 x 256 FP64 step 11.7 against 14.6 us
// with 256-wide tiles, FP32 the same).  PSCLBM_TILE_X in the environment (64,
// 128 or 256) overrides the choice, for measurements.
int tile_width(int nx, int nz) {
  if (const char* e = std::getenv("PSCLBM_TILE_X")) {
    const int v = std::atoi(e);
    if (v == 64 || v == 128 || v == 256) return v;
  }
  if (nz == 1) return 64;
  int best = 64;
  long long pad = ((long long)nx + 63) / 64 * 64;
  for (int tw : {128, 256}) {
    const long long p = ((long long)nx + tw - 1) / tw * tw;
    if (p <= pad) {
      best = tw;
      pad = p;
    }
  }
  return best;
}

// Even steps read and write every cell's own slots, each line by one wave
// only, and stream them with non-temporal hints when the distributions are
// larger than the 256 MB last-level cache (which they would otherwise sweep
// out).  PSCLBM_NT=0/1 overrides, for measurements.
int nt_even(const psclbm_config* c) {
  if (const char* e = std::getenv("PSCLBM_NT")) return std::atoi(e) ? 1 : 0;
  const double bytes = (double)c->nx * c->ny * c->nz * c->lattice * storage_bytes(c->precision);
  return bytes > 256.0 * 1024 * 1024 ? 1 : 0;
}

struct Layout {
  size_t f, err, scalar, tile_count, tile_list, snap, facc0, facc1, mass_part, outlet_u, outlet_g;
  size_t bin_count, bin_rec, cn0, cn1, cid0, cid1, fcont, spr0, spr1, ws0, ws1, total;
  int ntx, nty, ntz, ntiles, twx, twy;
  long long face_stride;
  int nbin[3];
  double bin_size[3];
  int bin_cap;
};

Layout plan(const psclbm_config* c) {
  Layout l;
  const long long N = (long long)c->nx * c->ny * c->nz;
  l.twx = tile_width(c->nx, c->nz);
  l.twy = BLOCK / l.twx;
  l.ntx = (c->nx + l.twx - 1) / l.twx;
  l.nty = (c->ny + l.twy - 1) / l.twy;
  l.ntz = c->nz;
  l.ntiles = l.ntx * l.nty * l.ntz;
  const int np = c->max_particles;
  const int cap = np > 0 ? c->max_tile_particles : 1;
  bool outlet = false;
  for (int f = 0; f < 6; ++f) outlet |= c->face_bc[f] == PSCLBM_OUTLET_EQ;
  long long fs = (long long)c->ny * c->nz;
  if ((long long)c->nx * c->nz > fs) fs = (long long)c->nx * c->nz;
  if ((long long)c->nx * c->ny > fs) fs = (long long)c->nx * c->ny;
  l.face_stride = fs;
  // DEM bins: at least 2 r_max + 1 wide so that every contact partner (centre
  // distance below r_i + r_j + delta_C with delta_C <= 1) is in a neighbour bin
  const int L[3] = {c->nx, c->ny, c->nz};
  const double bs = np > 0 ? 2.0 * c->max_radius + 1.0 : 1.0;
  for (int a = 0; a < 3; ++a) {
    if (a == 2 && c->lattice == 9) {
      l.nbin[a] = 1;
      l.bin_size[a] = 1.0;
      continue;
    }
    int nb = (int)std::floor(L[a] / bs);
    if (nb < 1) nb = 1;
    l.nbin[a] = nb;
    l.bin_size[a] = (double)L[a] / nb;
  }
  l.bin_cap = 32;
  const size_t nbins = (size_t)l.nbin[0] * l.nbin[1] * l.nbin[2];
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align_up(bytes > 0 ? bytes : 1);
    return at;
  };
  l.f = take((size_t)N * c->lattice * storage_bytes(c->precision));
  l.err = take(sizeof(unsigned) * 4);
  l.scalar = take(sizeof(double) * 4);
  l.tile_count = take(sizeof(int) * 2 * (size_t)l.ntiles);
  l.tile_list = take(sizeof(int) * (size_t)l.ntiles * cap);
  l.snap = take(sizeof(PSnap) * (size_t)(np > 0 ? np : 1));
  l.facc0 = take(sizeof(double) * 6 * (size_t)(np > 0 ? np : 1));
  l.facc1 = take(sizeof(double) * 6 * (size_t)(np > 0 ? np : 1));
  l.mass_part = take(sizeof(double) * (size_t)l.ntiles);
  l.outlet_u = take(outlet ? sizeof(double) * 3 * 6 * (size_t)fs : 8);
  l.outlet_g = take(outlet ? sizeof(double) * 3 * 6 * (size_t)fs : 8);
  const int mc = np > 0 ? c->max_contacts : 1;
  l.bin_count = take(sizeof(int) * 3 * nbins);
  l.bin_rec = take(sizeof(double) * 8 * 3 * nbins * l.bin_cap * (np > 0 ? 1 : 0));
  l.cn0 = take(sizeof(int) * (size_t)(np > 0 ? np : 1));
  l.cn1 = take(sizeof(int) * (size_t)(np > 0 ? np : 1));
  l.cid0 = take(sizeof(int) * (size_t)(np > 0 ? np : 1) * mc);
  l.cid1 = take(sizeof(int) * (size_t)(np > 0 ? np : 1) * mc);
  l.fcont = take(sizeof(double) * 3 * (size_t)(np > 0 ? np : 1));
  l.spr0 = take(sizeof(double) * SPRINGS * (size_t)(np > 0 ? np : 1) * mc);
  l.spr1 = take(sizeof(double) * SPRINGS * (size_t)(np > 0 ? np : 1) * mc);
  l.ws0 = take(sizeof(double) * 3 * (size_t)(np > 0 ? np : 1));
  l.ws1 = take(sizeof(double) * 3 * (size_t)(np > 0 ? np : 1));
  l.total = off;
  return l;
}

// The lattice geometry the kernels take, from a validated configuration.
void fill_geom(const psclbm_config* cfg, const Layout& l, Geom& g) {
  g.nx = cfg->nx;
  g.ny = cfg->ny;
  g.nz = cfg->nz;
  g.N = (long long)cfg->nx * cfg->ny * cfg->nz;
  g.q = cfg->lattice;
  for (int f = 0; f < 6; ++f) {
    g.face[f] = cfg->face_bc[f];
    if (cfg->lattice == 9 && f >= 4) g.face[f] = PSCLBM_PERIODIC;
    for (int k = 0; k < 3; ++k) g.face_u[f][k] = cfg->face_velocity[f][k];
  }
  for (int a = 0; a < 3; ++a) g.periodic[a] = axis_is_periodic(cfg, a) ? 1 : 0;
  g.ntx = l.ntx;
  g.nty = l.nty;
  g.ntz = l.ntz;
  g.twx = l.twx;
  g.twy = l.twy;
  g.remap = l.twx == SEG ? 1 : 0;
  g.nt_even = nt_even(cfg);
  g.rho0 = cfg->rho0;
}

int sticky(psclbm_ctx* c, bool clear) {
  unsigned bits = 0;
  int rc = hip_ok(hipMemcpyAsync(&bits, c->err, sizeof(unsigned), hipMemcpyDeviceToHost,
                                 c->stream));
  if (rc) return rc;
  rc = hip_ok(hipStreamSynchronize(c->stream));
  if (rc) return rc;
  if (bits && clear) {
    rc = hip_ok(hipMemsetAsync(c->err, 0, sizeof(unsigned), c->stream));
    if (rc) return rc;
  }
  if (bits & ERR_SLOTS) return PSCLBM_ESLOTS;
  if (bits & ERR_CONTACTS) return PSCLBM_ECONTACTS;
  if (bits & ERR_RADIUS) return PSCLBM_EINVAL;
  return PSCLBM_OK;
}

// ---------------------------------------------------------------------------
// Scratch of psc_solid_fraction_noalloc: one fixed device array per GPU,
// holding the error word, the tile counts, the tile lists, the particle
// snapshot and the force rows the rasterisation clears.  Host code reaches it
// only through the address hipGetSymbolAddress returns for the current
// device (the array's name is not a device address on the host).
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_BYTES = 32u << 20;
static_assert(NOALLOC_BYTES == (size_t)PSCLBM_NOALLOC_SCRATCH_BYTES, "scratch size of the header");
static __device__ __align__(256) __attribute__((used)) unsigned char scratch[NOALLOC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mutex;
void* scratch_ptr[MAX_DEVICES];

// The current device's address of the scratch array, looked up on its first
// use on that device (with that device current).
int scratch_address(void** out) {
  int dev = 0;
  int rc = hip_ok(hipGetDevice(&dev));
  if (rc) return rc;
  if (dev < 0 || dev >= MAX_DEVICES) return PSCLBM_EHIP;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    rc = hip_ok(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (rc) return rc;
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return PSCLBM_OK;
}

__global__ void k_zero_words(unsigned* p, long long n) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x)
    p[k] = 0u;
}

}  // namespace

extern "C" {

size_t psclbm_workspace_bytes(const psclbm_config* cfg) {
  if (validate(cfg) != PSCLBM_OK) return 0;
  return plan(cfg).total;
}

int lbm_init(const psclbm_config* cfg, void* d_workspace, size_t bytes, void* hip_stream,
             psclbm_ctx** out) {
  if (!out) return PSCLBM_EINVAL;
  *out = nullptr;
  int rc = validate(cfg);
  if (rc) return rc;
  if (!d_workspace || ((uintptr_t)d_workspace % ALIGN) != 0) return PSCLBM_EINVAL;
  const Layout l = plan(cfg);
  if (bytes < l.total) return PSCLBM_ENOMEM;
  psclbm_ctx* c = new (std::nothrow) psclbm_ctx();
  if (!c) return PSCLBM_EINVAL;
  std::memset(c, 0, sizeof(*c));
  c->cfg = *cfg;
  c->stream = static_cast<hipStream_t>(hip_stream);
  char* base = static_cast<char*>(d_workspace);
  fill_geom(cfg, l, c->geom);
  c->prec = cfg->precision;
  c->f = base + l.f;
  c->err = reinterpret_cast<unsigned*>(base + l.err);
  c->scalar = reinterpret_cast<double*>(base + l.scalar);
  c->tile_count_buf[0] = reinterpret_cast<int*>(base + l.tile_count);
  c->tile_count_buf[1] = c->tile_count_buf[0] + l.ntiles;
  c->tile_cur = 0;
  c->tile_count = c->tile_count_buf[0];
  c->tile_list = reinterpret_cast<int*>(base + l.tile_list);
  c->ntiles = l.ntiles;
  c->snap = reinterpret_cast<PSnap*>(base + l.snap);
  c->facc[0] = reinterpret_cast<double*>(base + l.facc0);
  c->facc[1] = reinterpret_cast<double*>(base + l.facc1);
  c->mass_part = reinterpret_cast<double*>(base + l.mass_part);
  c->nblocks = l.ntiles;
  c->outlet_u = reinterpret_cast<double*>(base + l.outlet_u);
  c->outlet_g = reinterpret_cast<double*>(base + l.outlet_g);
  c->face_stride = l.face_stride;
  for (int a = 0; a < 3; ++a) {
    c->nbin[a] = l.nbin[a];
    c->bin_size[a] = l.bin_size[a];
  }
  c->bin_cap = l.bin_cap;
  {
    const size_t nbins = (size_t)l.nbin[0] * l.nbin[1] * l.nbin[2];
    c->bin_count_buf[0] = reinterpret_cast<int*>(base + l.bin_count);
    c->bin_count_buf[1] = c->bin_count_buf[0] + nbins;
    c->bin_count_buf[2] = c->bin_count_buf[1] + nbins;
  }
  c->bin_cur = 0;
  {
    const size_t nrec = (size_t)l.nbin[0] * l.nbin[1] * l.nbin[2] * l.bin_cap * 8;
    for (int k = 0; k < 3; ++k)
      c->bin_rec[k] = reinterpret_cast<double*>(base + l.bin_rec) + (cfg->max_particles > 0 ? k * nrec : 0);
  }
  c->contact_n[0] = reinterpret_cast<int*>(base + l.cn0);
  c->contact_n[1] = reinterpret_cast<int*>(base + l.cn1);
  c->contact_id[0] = reinterpret_cast<int*>(base + l.cid0);
  c->contact_id[1] = reinterpret_cast<int*>(base + l.cid1);
  c->fcontact = reinterpret_cast<double*>(base + l.fcont);
  c->contact_springs[0] = reinterpret_cast<double*>(base + l.spr0);
  c->contact_springs[1] = reinterpret_cast<double*>(base + l.spr1);
  c->wsnap[0] = reinterpret_cast<double*>(base + l.ws0);
  c->wsnap[1] = reinterpret_cast<double*>(base + l.ws1);
  // clear everything but the distributions, then set f = f^eq(rho0, 0)
  rc = launch_zero(c, base + l.err, l.total - l.err);
  if (!rc) rc = launch_init_equilibrium(c, nullptr, nullptr);
  if (rc) {
    delete c;
    return rc;
  }
  *out = c;
  return PSCLBM_OK;
}

void lbm_free(psclbm_ctx* ctx) { delete ctx; }

int psclbm_set_stream(psclbm_ctx* ctx, void* hip_stream) {
  if (!ctx) return PSCLBM_EINVAL;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return PSCLBM_OK;
}

int lbm_set_f(psclbm_ctx* ctx, const double* d_f) {
  if (!ctx || !d_f) return PSCLBM_EINVAL;
  int rc = launch_set_f(ctx, d_f);
  if (rc) return rc;
  ctx->steps = 0;
  ctx->mass_valid = 0;
  return PSCLBM_OK;
}

int lbm_get_f(psclbm_ctx* ctx, double* d_f) {
  if (!ctx || !d_f) return PSCLBM_EINVAL;
  return launch_get_f(ctx, d_f);
}

int lbm_set_equilibrium(psclbm_ctx* ctx, const double* d_rho, const double* d_u) {
  if (!ctx) return PSCLBM_EINVAL;
  int rc = launch_init_equilibrium(ctx, d_rho, d_u);
  if (rc) return rc;
  ctx->steps = 0;
  ctx->mass_valid = 0;
  return PSCLBM_OK;
}

int lbm_get_macros(psclbm_ctx* ctx, double* d_rho, double* d_u) {
  if (!ctx) return PSCLBM_EINVAL;
  if (!d_rho && !d_u) return PSCLBM_OK;
  return launch_get_macros(ctx, d_rho, d_u);
}

int psc_rasterize(psclbm_ctx* ctx, const psclbm_particles* p) {
  if (!ctx || !p) return PSCLBM_EINVAL;
  if (p->n < 0 || p->n > ctx->cfg.max_particles) return PSCLBM_EINVAL;
  if (p->n > 0 && (!p->x || !p->u || !p->omega || !p->radius)) return PSCLBM_EINVAL;
  int rc = launch_rasterize(ctx, p, false);
  if (rc) return rc;
  ctx->np = p->n;
  ctx->rasterized = 1;
  return PSCLBM_OK;
}

int psc_get_solid_fraction(psclbm_ctx* ctx, double* d_eps_total, int* d_slot_id,
                           double* d_slot_eps, int kslots) {
  if (!ctx || kslots < 0) return PSCLBM_EINVAL;
  if (!ctx->rasterized) return PSCLBM_ESTATE;
  if (kslots == 0) d_slot_id = nullptr, d_slot_eps = nullptr;
  return launch_solid_fraction(ctx, d_eps_total, d_slot_id, d_slot_eps, kslots);
}

int lbm_step(psclbm_ctx* ctx, int nsteps) {
  if (!ctx || nsteps < 1) return PSCLBM_EINVAL;
  if (!ctx->rasterized) return PSCLBM_ESTATE;
  for (int k = 0; k < nsteps; ++k) {
    int rc = launch_step(ctx);
    if (rc) return rc;
  }
  return PSCLBM_OK;
}

int particle_forces(psclbm_ctx* ctx, double* d_force, double* d_torque) {
  if (!ctx) return PSCLBM_EINVAL;
  if (!ctx->rasterized) return PSCLBM_ESTATE;
  if (ctx->np == 0 || (!d_force && !d_torque)) return PSCLBM_OK;
  const double* src = ctx->facc[ctx->force_buf];
  const size_t pitch = 6 * sizeof(double);
  int rc = PSCLBM_OK;
  if (d_force)
    rc = hip_ok(hipMemcpy2DAsync(d_force, 3 * sizeof(double), src, pitch, 3 * sizeof(double),
                                 ctx->np, hipMemcpyDeviceToDevice, ctx->stream));
  if (!rc && d_torque)
    rc = hip_ok(hipMemcpy2DAsync(d_torque, 3 * sizeof(double), src + 3, pitch,
                                 3 * sizeof(double), ctx->np, hipMemcpyDeviceToDevice,
                                 ctx->stream));
  return rc;
}

// Material and friction parameters of a dynamic DEM step.
static bool dem_material_ok(const psclbm_dem_params* p) {
  if (!(p->rho_p > 0.0) || !(p->E_p > 0.0) || !(p->gamma >= 0.0) ||
      !(p->poisson > -1.0 && p->poisson < 0.5) || !(p->eta_n >= 0.0))
    return false;
  if (!(p->k_t >= 0.0) || !(p->eta_t >= 0.0) || !(p->mu_f >= 0.0) || !(p->theta_r >= 0.0) ||
      !std::isfinite(p->k_t) || !std::isfinite(p->eta_t) || !std::isfinite(p->mu_f) ||
      !std::isfinite(p->theta_r))
    return false;
  return p->mu_f == 0.0 || p->k_t > 0.0;  // the slider divides by k_T
}

int dem_step(psclbm_ctx* ctx, const psclbm_dem_params* prm, double* d_x, double* d_u,
             double* d_omega, const double* d_radius, int n, const double* d_force,
             const double* d_torque) {
  if (!ctx || !prm) return PSCLBM_EINVAL;
  if (n < 0 || n > ctx->cfg.max_particles) return PSCLBM_EINVAL;
  if (n == 0) return PSCLBM_OK;
  if (!d_x || !d_u || !d_omega || !d_radius) return PSCLBM_EINVAL;
  if ((d_force == nullptr) != (d_torque == nullptr)) return PSCLBM_EINVAL;
  if (!prm->kinematic && !d_force) {
    // use the accumulators of the most recent lbm_step (same particle count)
    if (!ctx->rasterized || n != ctx->np) return PSCLBM_ESTATE;
  }
  if (prm->n_sub < 1 || !(prm->dt > 0.0) || !std::isfinite(prm->dt)) return PSCLBM_EINVAL;
  if (!prm->kinematic && !dem_material_ok(prm)) return PSCLBM_EINVAL;
  return launch_dem_step(ctx, prm, d_x, d_u, d_omega, d_radius, n, d_force, d_torque);
}

int coupled_step(psclbm_ctx* ctx, const psclbm_dem_params* prm, double* d_x, double* d_u,
                 double* d_omega, const double* d_radius, int n, int nsteps) {
  if (!ctx || !prm || nsteps < 1) return PSCLBM_EINVAL;
  if (n < 0 || n > ctx->cfg.max_particles) return PSCLBM_EINVAL;
  if (n > 0 && (!d_x || !d_u || !d_omega || !d_radius)) return PSCLBM_EINVAL;
  if (prm->n_sub < 1 || !(prm->dt > 0.0) || !std::isfinite(prm->dt)) return PSCLBM_EINVAL;
  if (!prm->kinematic && !dem_material_ok(prm)) return PSCLBM_EINVAL;
  const int rc = launch_coupled(ctx, prm, d_x, d_u, d_omega, d_radius, n, nsteps);
  if (rc) return rc;
  ctx->np = n;
  ctx->rasterized = 1;
  return PSCLBM_OK;
}

int dem_step_adjoint(psclbm_ctx* ctx, const psclbm_dem_params* prm, const double* d_x,
                     const double* d_u, const double* d_omega, const double* d_radius, int n,
                     const double* d_gx, const double* d_gu, const double* d_gw, double* d_ax,
                     double* d_au, double* d_aw, double* d_aF, double* d_aT) {
  if (!ctx || !prm) return PSCLBM_EINVAL;
  if (n < 0 || n > ctx->cfg.max_particles) return PSCLBM_EINVAL;
  if (n == 0) return PSCLBM_OK;
  if (!d_x || !d_u || !d_omega || !d_radius || !d_gx || !d_gu || !d_gw || !d_ax || !d_au ||
      !d_aw || !d_aF || !d_aT)
    return PSCLBM_EINVAL;
  if (prm->kinematic || prm->n_sub != 1 || !(prm->dt > 0.0) || !std::isfinite(prm->dt) ||
      !dem_material_ok(prm) || prm->mu_f != 0.0 || prm->theta_r != 0.0)
    return PSCLBM_EINVAL;
  return launch_dem_adjoint(ctx, prm, d_x, d_u, d_radius, n, d_gx, d_gu, d_gw, d_ax, d_au, d_aw,
                            d_aF, d_aT);
}

int dem_reset_contacts(psclbm_ctx* ctx) {
  if (!ctx) return PSCLBM_EINVAL;
  return launch_dem_reset(ctx);
}

int dem_get_contacts(psclbm_ctx* ctx, int* d_count, int* d_ids) {
  if (!ctx || !d_count || !d_ids) return PSCLBM_EINVAL;
  const size_t np = (size_t)ctx->cfg.max_particles;
  if (np == 0) return PSCLBM_OK;
  const size_t mc = (size_t)ctx->cfg.max_contacts;
  int rc = hip_ok(hipMemcpyAsync(d_count, ctx->contact_n[ctx->contact_cur], sizeof(int) * np,
                                 hipMemcpyDeviceToDevice, ctx->stream));
  if (!rc)
    rc = hip_ok(hipMemcpyAsync(d_ids, ctx->contact_id[ctx->contact_cur], sizeof(int) * np * mc,
                               hipMemcpyDeviceToDevice, ctx->stream));
  return rc;
}

int dem_set_contacts(psclbm_ctx* ctx, const int* d_count, const int* d_ids) {
  if (!ctx || !d_count || !d_ids) return PSCLBM_EINVAL;
  const size_t np = (size_t)ctx->cfg.max_particles;
  if (np == 0) return PSCLBM_OK;
  const size_t mc = (size_t)ctx->cfg.max_contacts;
  int rc = hip_ok(hipMemcpyAsync(ctx->contact_n[ctx->contact_cur], d_count, sizeof(int) * np,
                                 hipMemcpyDeviceToDevice, ctx->stream));
  if (!rc)
    rc = hip_ok(hipMemcpyAsync(ctx->contact_id[ctx->contact_cur], d_ids, sizeof(int) * np * mc,
                               hipMemcpyDeviceToDevice, ctx->stream));
  ctx->springs_valid = 0;  // springs are not part of the saved lists
  return rc;
}

int lbm_mass(psclbm_ctx* ctx, double* h_mass) {
  if (!ctx || !h_mass) return PSCLBM_EINVAL;
  int rc = launch_mass(ctx, h_mass);
  if (rc) return rc;
  rc = sticky(ctx, true);
  if (rc) return rc;
  if (!std::isfinite(*h_mass)) return PSCLBM_ENONFINITE;
  return PSCLBM_OK;
}

int psclbm_sync(psclbm_ctx* ctx) {
  if (!ctx) return PSCLBM_EINVAL;
  return sticky(ctx, true);
}

long long lbm_step_count(const psclbm_ctx* ctx) { return ctx ? ctx->steps : -1; }

int lbm_step_adjoint(psclbm_ctx* ctx, const double* d_f, const double* d_lambda_in,
                     double* d_lambda_out, const double* d_dJ_dF, const double* d_dJ_dT,
                     double* d_g_x, double* d_g_u, double* d_g_omega,
                     double* d_g_face_velocity) {
  if (!ctx || !d_f || !d_lambda_in || !d_lambda_out) return PSCLBM_EINVAL;
  if (d_lambda_in == d_lambda_out) return PSCLBM_EINVAL;
  if (ctx->cfg.weighting != PSCLBM_WEIGHT_MODIFIED) return PSCLBM_EINVAL;
  if (!ctx->rasterized) return PSCLBM_ESTATE;
  return launch_adjoint(ctx, d_f, d_lambda_in, d_lambda_out, d_dJ_dF, d_dJ_dT, d_g_x, d_g_u,
                        d_g_omega, d_g_face_velocity);
}

int lbm_recompute(psclbm_ctx* ctx, const double* d_f0, int nsteps, double* d_ring) {
  if (!ctx || !d_f0 || !d_ring || nsteps < 1) return PSCLBM_EINVAL;
  if (!ctx->rasterized) return PSCLBM_ESTATE;
  // the ring step addresses one direction's FP64 array with 32-bit byte offsets
  if ((double)ctx->geom.N * sizeof(double) >= 4294967296.0) return PSCLBM_EINVAL;
  const size_t QN = (size_t)ctx->geom.q * (size_t)ctx->geom.N;
  const uintptr_t r0 = (uintptr_t)d_ring, r1 = r0 + (uintptr_t)nsteps * QN * sizeof(double);
  const uintptr_t f0 = (uintptr_t)d_f0, f1 = f0 + QN * sizeof(double);
  if (f0 < r1 && r0 < f1) return PSCLBM_EINVAL;
  return launch_recompute(ctx, d_f0, nsteps, d_ring);
}

int psc_rasterize_adjoint(psclbm_ctx* ctx, const double* d_g_slot_eps, int kslots,
                          double* d_g_x) {
  if (!ctx || !d_g_slot_eps || !d_g_x || kslots < 1) return PSCLBM_EINVAL;
  if (!ctx->rasterized) return PSCLBM_ESTATE;
  if (ctx->np == 0) return PSCLBM_OK;
  return launch_rasterize_adjoint(ctx, d_g_slot_eps, kslots, d_g_x);
}

int psc_solid_fraction_noalloc(const psclbm_config* cfg, const psclbm_particles* p,
                               double* d_eps_total, int* d_slot_id, double* d_slot_eps,
                               int kslots, void* hip_stream) {
  if (!cfg || !p || !d_eps_total || kslots < 0) return PSCLBM_EINVAL;
  int rc = validate(cfg);
  if (rc) return rc;
  if (cfg->max_particles < 1 || p->n < 0 || p->n > cfg->max_particles) return PSCLBM_EINVAL;
  if (p->n > 0 && (!p->x || !p->u || !p->omega || !p->radius)) return PSCLBM_EINVAL;
  if (kslots > 0 && (!d_slot_id || !d_slot_eps)) return PSCLBM_EINVAL;
  const Layout l = plan(cfg);
  const int np = p->n > 0 ? p->n : 1;
  // the scratch layout: error word, two sets of tile counts, tile lists,
  // snapshot, one block of force rows (cleared by the rasterisation)
  const size_t o_err = 0;
  const size_t o_cnt = align_up(sizeof(unsigned));
  const size_t o_list = o_cnt + align_up(sizeof(int) * 2 * (size_t)l.ntiles);
  const size_t o_snap = o_list + align_up(sizeof(int) * (size_t)l.ntiles * cfg->max_tile_particles);
  const size_t o_facc = o_snap + align_up(sizeof(PSnap) * (size_t)np);
  const size_t need = o_facc + align_up(sizeof(double) * 6 * (size_t)np);
  if (need > NOALLOC_BYTES) return PSCLBM_EINVAL;
  void* sp = nullptr;
  rc = scratch_address(&sp);
  if (rc) return rc;
  char* base = static_cast<char*>(sp);
  psclbm_ctx c;
  std::memset(&c, 0, sizeof(c));
  c.cfg = *cfg;
  c.stream = static_cast<hipStream_t>(hip_stream);
  fill_geom(cfg, l, c.geom);
  c.err = reinterpret_cast<unsigned*>(base + o_err);
  c.tile_count_buf[0] = reinterpret_cast<int*>(base + o_cnt);
  c.tile_count_buf[1] = c.tile_count_buf[0] + l.ntiles;
  c.tile_cur = 0;
  c.tile_count = c.tile_count_buf[0];
  c.tile_list = reinterpret_cast<int*>(base + o_list);
  c.ntiles = l.ntiles;
  c.snap = reinterpret_cast<PSnap*>(base + o_snap);
  c.facc[0] = c.facc[1] = reinterpret_cast<double*>(base + o_facc);
  // the array keeps the last call's contents: clear the error word and the
  // tile counts with a kernel (no memset node, no allocation)
  const long long words = (long long)(o_list / sizeof(unsigned));
  k_zero_words<<<(unsigned)((words + 255) / 256 < 4096 ? (words + 255) / 256 : 4096), 256, 0,
                 c.stream>>>(reinterpret_cast<unsigned*>(base), words);
  rc = hip_ok(hipGetLastError());
  if (!rc) rc = launch_rasterize(&c, p, false);
  if (rc) return rc;
  c.np = p->n;
  rc = launch_solid_fraction(&c, d_eps_total, kslots > 0 ? d_slot_id : nullptr,
                             kslots > 0 ? d_slot_eps : nullptr, kslots);
  if (rc) return rc;
  return sticky(&c, false);
}

const char* psclbm_strerror(int code) {
  switch (code) {
    case PSCLBM_OK: return "success";
    case PSCLBM_EINVAL: return "invalid argument or configuration";
    case PSCLBM_ENOMEM: return "workspace smaller than psclbm_workspace_bytes()";
    case PSCLBM_EHIP: return "HIP runtime error";
    case PSCLBM_ESLOTS: return "a cell or tile particle list exceeded its capacity";
    case PSCLBM_ECONTACTS: return "DEM contact list or bin exceeded its capacity";
    case PSCLBM_ENONFINITE: return "lattice mass is not finite";
    case PSCLBM_ESTATE: return "call out of order";
    default: return "unknown error";
  }
}

}  // extern "C"
