// Internal declarations of the gfx950 PSC-LBM library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "psclbm.h"

namespace psclbm {

// ---------------------------------------------------------------------------
// Lattice velocity sets in the canonical order of psclbm.h.
// ---------------------------------------------------------------------------
template <int Q>
struct Lattice;

template <>
struct Lattice<9> {
  static constexpr int D = 2;
  __host__ __device__ static constexpr int ex(int i) {
    return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0);
  }
  __host__ __device__ static constexpr int ey(int i) {
    return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0);
  }
  __host__ __device__ static constexpr int ez(int) { return 0; }
  // 1 <-> 3, 2 <-> 4, 5 <-> 7, 6 <-> 8
  __host__ __device__ static constexpr int opp(int i) {
    return i == 0 ? 0 : (i <= 4 ? (i + 1) % 4 + 1 : (i - 3) % 4 + 5);
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
};

template <>
struct Lattice<19> {
  static constexpr int D = 3;
  // rest, +-x, +-y, +-z, then the 12 edge vectors in (v, -v) pairs
  __host__ __device__ static constexpr int ex(int i) {
    return i == 1 || i == 7 || i == 9 || i == 11 || i == 13
               ? 1
               : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14 ? -1 : 0);
  }
  __host__ __device__ static constexpr int ey(int i) {
    return i == 3 || i == 7 || i == 10 || i == 15 || i == 17
               ? 1
               : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18 ? -1 : 0);
  }
  __host__ __device__ static constexpr int ez(int i) {
    return i == 5 || i == 11 || i == 14 || i == 15 || i == 18
               ? 1
               : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17 ? -1 : 0);
  }
  __host__ __device__ static constexpr int opp(int i) { return i == 0 ? 0 : (i % 2 ? i + 1 : i - 1); }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
};

// Storage / compute type pairs of the three precision forms.
template <int PREC>
struct Form;
template <>
struct Form<PSCLBM_FP64> {
  using S = double;  // stores f_i
  using C = double;
};
template <>
struct Form<PSCLBM_FP32> {
  using S = float;  // stores f_i - w_i rho0
  using C = float;
};
template <>
struct Form<PSCLBM_FP32_FP16STORE> {
  using S = _Float16;  // stores (f_i - w_i rho0) / w_i
  using C = float;
};

// Workgroup tile: 256 cells, twx along x by twy = 256 / twx rows along y (twx
// 64, 128 or 256, chosen per lattice), worked by four waves; each wave takes
// one 64-cell segment of one row.
constexpr int SEG = 64;
constexpr int BLOCK = 256;
constexpr int KSLOTS = 4;  // particles a single cell can be covered by

// Sticky device error bits.
constexpr unsigned ERR_SLOTS = 1u;
constexpr unsigned ERR_RADIUS = 2u;
constexpr unsigned ERR_CONTACTS = 4u;

// Snapshot of one particle used by the lattice kernels (FP64).
struct alignas(16) PSnap {
  double x[3];
  double r;
  double cs;  // V_a(r) + 1/2 (Eqs. 15, 18)
  double u[3];
  double w[3];
  double pad;
};

// Geometry shared by all lattice kernels (passed by value).
struct Geom {
  int nx, ny, nz;
  long long N;
  int q;
  int face[6];
  int periodic[3];
  int ntx, nty, ntz;
  int twx, twy;  // tile extent along x and y (twx * twy == BLOCK)
  int remap;     // deal the tiles to the XCDs in contiguous runs
  int nt_even;   // even steps stream the lattice with non-temporal loads and stores
  double face_u[6][3];
  double rho0;
};

// Doubles of friction springs kept per contact: the tangential displacement
// xi[3], the twist angle, the rolling displacement xr[3], one unused.
constexpr int SPRINGS = 8;

// Contact-pass arguments: the binning it reads and the contact lists.
struct DemArgs {
  int n;
  int three_d;
  int L[3];
  int periodic[3];
  int nbin[3];
  double bin_size[3];
  int bin_cap;
  const int* bin_count;  // counts of the current binning
  const double* bin_rec; // its records: x, u, r, id at the start of the sub-step
  const int* prev_n;
  const int* prev_id;
  int* next_n;
  int* next_id;
  int max_contacts;
  double E;       // effective modulus of two bodies of the material (Eq. 25)
  double gamma;
  double eta_n;
  unsigned* err;
};

struct StepArgs {
  Geom g;
  void* f;
  double tau;
  double force[3];
  double h;
  int np;
  int cap;                 // tile list capacity
  const int* tile_count;
  const int* tile_list;
  const PSnap* snap;
  double* facc;            // force / torque buffer accumulated this step: [np][6]
  double* fzero;           // the other buffer, cleared this step
  double* mass_part;       // per-block mass partials
  const double* outlet_u;  // [6][max face cells][3]
  long long face_stride;   // cells per face slot in outlet_u
  unsigned* err;
  double omega;            // 1 / tau
  double inv_rho0;         // 1 / rho0
  // the same uniform values rounded to FP32 for the FP32 arithmetic forms
  float force_f[3], omega_f, inv_rho0_f, rho0_f, tm_f;  // tm = tau - 1/2
  unsigned inlet_mask;     // faces of kind INLET_EQ (bit f)
  unsigned outlet_mask;    // faces of kind OUTLET_EQ
  unsigned open_mask;      // inlet | outlet
  unsigned moving_mask;    // faces of kind MOVING_WALL
  unsigned outlet_wave;    // outlet faces served from the neighbour's lane
  int original;            // original weighting (Eqs. 7-9, 11) instead of Eqs. 12-14
  const void* src;         // ring step: canonical FP64 state read (f is written)
  // coupled step: the leading dem_blocks workgroups gather the DEM contacts
  // of four particles each (positions px, velocities pu, radii pr at the
  // start of the step) into fc [n][3]; the tiles follow
  int dem_blocks;
  DemArgs dem;
  const double* px;
  const double* pu;
  const double* pr;
  double* fc;
};

// Outlet faces whose cells share a wave with their interior neighbour, so that
// the neighbour's velocity (and, in the adjoint, the sensitivity flowing back
// to it) moves between lanes: the x faces, since a wave is one 64-cell x-row
// segment (segments start at multiples of 64); x = nx-1 only when it is not
// the first lane of a segment.
inline unsigned outlet_wave_mask(const Geom& g, unsigned outlet_mask) {
  unsigned m = 0;
  if ((outlet_mask & 1u) && g.nx >= 2) m |= 1u;
  if ((outlet_mask & 2u) && g.nx >= 2 && (g.nx - 1) % SEG != 0) m |= 2u;
  return m;
}

}  // namespace psclbm

struct psclbm_ctx {
  psclbm_config cfg;
  hipStream_t stream;
  psclbm::Geom geom;
  int prec;
  void* f;
  unsigned* err;
  int* tile_count;          // counts of the current tile lists (one of tile_count_buf)
  int* tile_count_buf[2];    // double-buffered: each rasterisation clears the other
  int tile_cur;
  int* tile_list;
  int ntiles;
  psclbm::PSnap* snap;
  double* facc[2];
  double* mass_part;
  int nblocks;
  double* outlet_u;
  double* outlet_g;  // adjoint: dJ/du of each outlet cell's reset velocity
  long long face_stride;
  // DEM
  int nbin[3];
  double bin_size[3];
  int bin_cap;
  int* bin_count_buf[3];  // each binning fills set cur+1 and clears set cur+2
  double* bin_rec[3];     // per set: [bin][slot][8] = x, u, r, id of the entry
  int bin_cur;            // the set of the latest binning
  int* contact_n[2];
  int* contact_id[2];
  int contact_cur;
  double* fcontact;  // [max_particles][3] contact forces of the coupled step
  double* contact_springs[2];  // per contact list: [max_particles][max_contacts][SPRINGS]
  int springs_valid;           // the current list's springs were written (friction was on)
  double* wsnap[2];            // [max_particles][3] spins at the start of a friction (sub-)step;
                               // the fused coupled step alternates the two
  double* scalar;  // one FP64 device scalar for reductions
  // host-side state
  long long steps;
  int np;
  int rasterized;
  int force_buf;   // buffer holding the last step's forces
  int mass_valid;  // mass partials describe the current state
};

namespace psclbm {
// e . v for a lattice vector e with components in {-1, 0, 1} known at
// compile time after unrolling: only the nonzero components are summed, as
// the compiler may not drop 0 * v (IEEE), and +-1 * v is exact.
template <typename T>
__device__ __forceinline__ T edot(int ex, int ey, int ez, T a, T b, T c) {
  if (ex != 0) {
    T r = ex > 0 ? a : -a;
    if (ey != 0) r = ey > 0 ? r + b : r - b;
    if (ez != 0) r = ez > 0 ? r + c : r - c;
    return r;
  }
  if (ey != 0) {
    T r = ey > 0 ? b : -b;
    if (ez != 0) r = ez > 0 ? r + c : r - c;
    return r;
  }
  if (ez != 0) return ez > 0 ? c : -c;
  return T(0);
}

// acc += e v for a lattice component e in {-1, 0, 1}.
template <typename T>
__device__ __forceinline__ void eacc(int e, T& acc, T v) {
  if (e > 0) acc += v;
  if (e < 0) acc -= v;
}

// Target of a DEM binning: the count set to fill (all zero on entry), the set
// to clear for the binning after next, and the records of the filled set:
// each binned particle's position, velocity, radius and id, which the contact
// pass of that binning reads.
struct DemBinOut {
  int* count;  // null: no DEM binning
  int* stale;
  long long nbins;
  double* rec;
  int bin_cap;
  int nbin[3];
  double bin_size[3];
};

inline DemBinOut dem_bin_out(const psclbm_ctx* c, bool on) {
  DemBinOut b;
  const int fill = (c->bin_cur + 1) % 3;
  b.count = on ? c->bin_count_buf[fill] : nullptr;
  b.stale = c->bin_count_buf[(c->bin_cur + 2) % 3];
  b.nbins = on ? (long long)c->nbin[0] * c->nbin[1] * c->nbin[2] : 0;
  b.rec = c->bin_rec[fill];
  b.bin_cap = c->bin_cap;
  for (int a = 0; a < 3; ++a) {
    b.nbin[a] = c->nbin[a];
    b.bin_size[a] = c->bin_size[a];
  }
  return b;
}

// After a launch that binned through dem_bin_out: its set becomes current.
inline void dem_bins_advance(psclbm_ctx* c) { c->bin_cur = (c->bin_cur + 1) % 3; }

// Sum of a double over the 64 lanes of a wave with DPP lane moves (no LDS
// traffic): pairs and quads by quad permutes, rows of 16 by row shifts, then
// row broadcasts 15 and 31 carry the row totals up to lane 63, whose value is
// read back as a wave-uniform scalar.  Every lane of the wave must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ int dpp_move(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}

// Butterfly over aligned lane blocks of 2, 4 and 8 (DPP quad_perm [1,0,3,2],
// quad_perm [2,3,0,1], row_half_mirror): a block merges with its partner
// block when both hold one key (>= 0) throughout.  merge_flags gives the
// merge decision of each level (bit l of the result) and whether this lane
// leads its final block; merge_sum then sums a value over the final block.
// Every lane of the wave must be active.
__device__ __forceinline__ unsigned merge_flags(int key, int lane, bool& lead) {
  int uni = key >= 0 ? 1 : 0;
  unsigned m = 0;
  lead = key >= 0;
  {
    const bool mm = uni && dpp_move<0xB1>(uni) && key == dpp_move<0xB1>(key);
    m |= mm ? 1u : 0u;
    if (mm && (lane & 1)) lead = false;
    uni = mm ? 1 : 0;
  }
  {
    const bool mm = uni && dpp_move<0x4E>(uni) && key == dpp_move<0x4E>(key);
    m |= mm ? 2u : 0u;
    if (mm && (lane & 2)) lead = false;
    uni = mm ? 1 : 0;
  }
  {
    const bool mm = uni && dpp_move<0x141>(uni) && key == dpp_move<0x141>(key);
    m |= mm ? 4u : 0u;
    if (mm && (lane & 4)) lead = false;
  }
  return m;
}
template <typename T>
__device__ __forceinline__ T merge_sum(T v, unsigned m) {
  T w = dpp_move<0xB1>(v);
  if (m & 1u) v += w;
  w = dpp_move<0x4E>(v);
  if (m & 2u) v += w;
  w = dpp_move<0x141>(v);
  if (m & 4u) v += w;
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x114>(v);  // row_shr:4
  v += dpp_move<0x118>(v);  // row_shr:8
  v += dpp_move<0x142>(v);  // row_bcast:15
  v += dpp_move<0x143>(v);  // row_bcast:31
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Lanes of the wave below this one whose bit is set in mask.
__device__ __forceinline__ int lanes_below(unsigned long long mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Launchers (return a psclbm error code).
int launch_init_equilibrium(psclbm_ctx* c, const double* rho, const double* u);
int launch_set_f(psclbm_ctx* c, const double* f);
int launch_get_f(psclbm_ctx* c, double* f);
int launch_get_macros(psclbm_ctx* c, double* rho, double* u);
int launch_rasterize(psclbm_ctx* c, const psclbm_particles* p, bool dem_bins);
// The step with the contact workgroups of dem (the DEM contact forces of the
// step's start into fcontact); dem null: the plain step.
int launch_step_contacts(psclbm_ctx* c, const DemArgs* dem, const double* x, const double* u,
                         const double* r);
int launch_coupled(psclbm_ctx* c, const psclbm_dem_params* prm, double* x, double* u, double* w,
                   const double* r, int n, int nsteps);
int launch_solid_fraction(psclbm_ctx* c, double* eps, int* ids, double* seps, int k);
int launch_step(psclbm_ctx* c);
int launch_recompute(psclbm_ctx* c, const double* f0, int nsteps, double* ring);
int launch_mass(psclbm_ctx* c, double* h_mass);
int launch_zero(psclbm_ctx* c, void* p, size_t bytes);
int launch_dem_step(psclbm_ctx* c, const psclbm_dem_params* prm, double* x, double* u,
                    double* w, const double* r, int n, const double* F, const double* T);
int launch_dem_reset(psclbm_ctx* c);
int launch_adjoint(psclbm_ctx* c, const double* f, const double* lam_in, double* lam_out,
                   const double* gF, const double* gT, double* gX, double* gU, double* gW,
                   double* gface);
int launch_rasterize_adjoint(psclbm_ctx* c, const double* gs, int kslots, double* gX);
inline int hip_ok(hipError_t e) { return e == hipSuccess ? PSCLBM_OK : PSCLBM_EHIP; }
}  // namespace psclbm
