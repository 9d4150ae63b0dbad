// Lattice kernels of the gfx950 PSC-LBM library.
//
// Storage: one structure-of-arrays distribution array A[i][n] (n = x + nx*(y +
// ny*z)) updated in place with the two-parity "AA" streaming pattern, so each
// time step reads and writes every population exactly once:
//   even step (parity 0): cell n reads A[i][n] and writes its post-collision
//                          f*_i to A[opp(i)][n];
//   odd step  (parity 1): cell n reads f_i from A[opp(i)][n - e_i] and writes
//                          f*_i to A[i][n + e_i].
// A third form (ring step, used to recompute states for the adjoint) reads a
// canonical FP64 array and writes the canonical result into another:
//   ring step (parity 2): cell n reads src[i][n] and writes f*_i to dst[i][n + e_i].
// A link that leaves the domain through a non-periodic face is reflected into
// the cell itself (halfway bounce-back, Eq. 6), which in both parities lands
// on the location the same cell reads back next step; every location is read
// and written by one thread per step, so the update needs no second copy.
//
// Per-cell physics (Sec. 2.1-2.3): moments with the half-force shift (Eq. 5),
// BGK with Guo forcing (Eqs. 2-4), and in cells covered by particles the
// modified partially-saturated-cell collision (Eqs. 10, 12, 13) with the
// per-particle momentum exchange of Eq. 14.  The solid fractions (Eqs. 15-19,
// Table 1) are evaluated per cell from the workgroup tile's particle list held
// in LDS, so no per-cell solid data is stored in HBM.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <type_traits>

#include "common.hpp"
#include "dem.hpp"
#include "tiles.hpp"

namespace psclbm {

static_assert(Lattice<9>::opp(1) == 3 && Lattice<9>::opp(6) == 8 && Lattice<9>::opp(7) == 5,
              "D2Q9 opposite table");

template <int Q>
__host__ __device__ constexpr bool check_lattice() {
  for (int i = 0; i < Q; ++i) {
    const int o = Lattice<Q>::opp(i);
    if (Lattice<Q>::ex(o) != -Lattice<Q>::ex(i) || Lattice<Q>::ey(o) != -Lattice<Q>::ey(i) ||
        Lattice<Q>::ez(o) != -Lattice<Q>::ez(i))
      return false;
  }
  return true;
}
static_assert(check_lattice<9>() && check_lattice<19>(), "opposite directions");

// ---------------------------------------------------------------------------
// FP32 arithmetic that keeps the collision free of systematic rounding.
// ---------------------------------------------------------------------------
// w_i x in the compute type.  In FP32 the weights are not representable: 4/9,
// 1/9, 1/18 and 1/36 all round with one relative error of about 7.5e-9 (1/3
// with 3e-8), which scales the mass and momentum of every equilibrium the
// collision relaxes towards, and the relaxation then adds that excess to the
// flow again at every step.  The product is taken with the weight split into
// its FP32 rounding and the remainder, so that it carries one ordinary
// rounding of the result instead.
template <int Q, typename C>
__device__ __forceinline__ C wmul(int i, C x) {
  if constexpr (std::is_same<C, double>::value) {
    return (C)Lattice<Q>::w(i) * x;
  } else {
    const float hi = (float)Lattice<Q>::w(i);
    const float lo = (float)(Lattice<Q>::w(i) - (double)hi);
    return __builtin_fmaf(x, hi, x * lo);
  }
}

// The FP16 storage form keeps a cell's populations in registers as it stores
// them, h_i = g_i / w_i: the collision then takes no weight per direction,
// and the weights enter the moments once per weight class.
template <int PREC>
constexpr bool scaled_form() {
  return PREC == PSCLBM_FP32_FP16STORE;
}
// w_i x, or x itself in the scaled form
template <int Q, bool SC, typename C>
__device__ __forceinline__ C wq(int i, C x) {
  if constexpr (SC) return x;
  else return wmul<Q>(i, x);
}
// The density deviation sum_i g_i and the momentum sum_i e_i g_i of a cell;
// in the scaled form as sum_c w_c (sums over the rest, axis and diagonal
// classes of h_i).
template <int Q, bool SC, typename C>
__device__ __forceinline__ void cell_moments(const C (&g)[Q], C& r, C& jx, C& jy, C& jz) {
  using L = Lattice<Q>;
  if constexpr (!SC) {
    r = jx = jy = jz = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      r += g[i];
      if (L::ex(i) > 0) jx += g[i];
      if (L::ex(i) < 0) jx -= g[i];
      if (L::ey(i) > 0) jy += g[i];
      if (L::ey(i) < 0) jy -= g[i];
      if (L::ez(i) > 0) jz += g[i];
      if (L::ez(i) < 0) jz -= g[i];
    }
  } else {
    C R[3] = {0, 0, 0}, X[3] = {0, 0, 0}, Y[3] = {0, 0, 0}, Z[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int c = L::ex(i) * L::ex(i) + L::ey(i) * L::ey(i) + L::ez(i) * L::ez(i);
      R[c] += g[i];
      if (L::ex(i) > 0) X[c] += g[i];
      if (L::ex(i) < 0) X[c] -= g[i];
      if (L::ey(i) > 0) Y[c] += g[i];
      if (L::ey(i) < 0) Y[c] -= g[i];
      if (L::ez(i) > 0) Z[c] += g[i];
      if (L::ez(i) < 0) Z[c] -= g[i];
    }
    constexpr int axis = 1, diag = Q == 9 ? 5 : 7;  // a direction of each class
    r = wmul<Q>(0, R[0]) + (wmul<Q>(axis, R[1]) + wmul<Q>(diag, R[2]));
    jx = wmul<Q>(axis, X[1]) + wmul<Q>(diag, X[2]);
    jy = wmul<Q>(axis, Y[1]) + wmul<Q>(diag, Y[2]);
    jz = wmul<Q>(axis, Z[1]) + wmul<Q>(diag, Z[2]);
  }
}

// Velocity of Eq. 5, u = (j + F/2) / rho, in the compute type, from the
// momentum component j, the half force h and q = drho / rho.  In FP32 the half
// force (of order 1e-7 against a momentum of order 1e-3 in a slowly developing
// flow) loses its low bits when added to j, the same bits step after step,
// which biases the force the flow receives; the sum is therefore kept as its
// rounded value s and the exact remainder e (Knuth's two-sum), and 1/rho as
// (1 - q) / rho0, so that the rounding of rho only touches the small
// correction: u = (s + (e - s q)) / rho0.
template <typename C>
__device__ __forceinline__ C eq5_velocity(C j, C h, C q, C inv_rho, C inv_rho0) {
  if constexpr (std::is_same<C, double>::value) {
    (void)q;
    (void)inv_rho0;
    return (j + h) * inv_rho;
  } else {
    (void)inv_rho;
    const C s = j + h;
    const C bp = s - j;
    const C e = (j - (s - bp)) + (h - bp);
    return (s + (e - s * q)) * inv_rho0;
  }
}

// The same without a body force: the sum j + F/2 is j itself, so the FP32
// form is one fused multiply-add, u = (j - j q) / rho0.
template <typename C>
__device__ __forceinline__ C eq5_velocity_unforced(C j, C q, C inv_rho, C inv_rho0) {
  if constexpr (std::is_same<C, double>::value) {
    (void)q;
    (void)inv_rho0;
    return j * inv_rho;
  } else {
    (void)inv_rho;
    return __builtin_fmaf(-j, q, j) * inv_rho0;
  }
}

// 1/rho for Eq. 5: exact in FP64. The FP32 forms use it only for q = drho /
// rho, the small correction in both velocities above, where the hardware
// reciprocal's last bit stays below the velocity's own rounding.
template <typename C>
__device__ __forceinline__ C inv_density(C rho) {
  if constexpr (std::is_same<C, double>::value) return 1.0 / rho;
  else return __builtin_amdgcn_rcpf(rho);
}

// ---------------------------------------------------------------------------
// Storage conversion: deviation g_i = f_i - w_i rho0 in the compute type (in
// the FP16 form g_i / w_i, as stored).
// ---------------------------------------------------------------------------
// Direction i's array of a state with N cells, as a base the compiler holds
// in scalar registers and cannot re-derive from the others. Where all Q
// accesses of a cell share one offset (the even step's own-cell accesses) it
// otherwise forms each 64-bit address with a vector add from the previous one.
template <typename S>
__device__ __forceinline__ S* dir_ptr(S* A, int i, unsigned N) {
  S* p = A + (size_t)i * N;
  asm("" : "+s"(p));
  return p;
}
// Element `e` of a per-direction array through a 32-bit byte offset, in the
// global address space, so the access is the scalar base plus one 32-bit
// vector offset.
template <typename S>
using GlobalT = __attribute__((address_space(1))) S;
template <typename S>
__device__ __forceinline__ GlobalT<S>& elem(S* base, unsigned e) {
  auto* gb = (__attribute__((address_space(1))) char*)base;
  return *(GlobalT<S>*)(gb + (e * (unsigned)sizeof(S)));
}
// The same element read or written with a non-temporal hint when NT: the
// line is streamed through the caches rather than kept in them.
template <bool NT, typename S>
__device__ __forceinline__ S elem_ld(S* base, unsigned e) {
  if constexpr (NT) return __builtin_nontemporal_load(&elem(base, e));
  else return elem(base, e);
}
template <bool NT, typename S>
__device__ __forceinline__ void elem_st(S* base, unsigned e, S v) {
  if constexpr (NT) __builtin_nontemporal_store(v, &elem(base, e));
  else elem(base, e) = v;
}

template <int PREC, int Q>
struct Store {
  using S = typename Form<PREC>::S;
  using C = typename Form<PREC>::C;
  // direction-i array `b` (= A + i N), element e: the deviation g_i in the
  // compute type, or g_i / w_i as stored in the scaled (FP16) form
  template <bool NT = false>
  __device__ static C ld(S* b, unsigned e, int i, double rho0) {
    const S v = elem_ld<NT>(b, e);
    if constexpr (PREC == PSCLBM_FP64) {
      return v - Lattice<Q>::w(i) * rho0;
    } else if constexpr (PREC == PSCLBM_FP32) {
      return v;
    } else {
      (void)i;
      return static_cast<float>(v);
    }
  }
  // stores deviation g of direction i (g / w_i in the scaled form); returns
  // the deviation memory now holds in FP64 (exactly, and in the FP16 form to
  // the rounding of h w_i: the per-cell part of the mass sum)
  template <bool NT = false>
  __device__ static double st(S* b, unsigned e, int i, C g, double rho0) {
    if constexpr (PREC == PSCLBM_FP64) {
      const double f = Lattice<Q>::w(i) * rho0 + g;
      elem_st<NT>(b, e, f);
      return f - Lattice<Q>::w(i) * rho0;
    } else if constexpr (PREC == PSCLBM_FP32) {
      elem_st<NT>(b, e, g);
      return static_cast<double>(g);
    } else {
      const _Float16 h = static_cast<_Float16>(g);
      elem_st<NT>(b, e, h);
      return static_cast<double>(static_cast<float>(h)) * Lattice<Q>::w(i);
    }
  }
  // Exact canonical FP64 value of stored population i.
  __device__ static double to_f64(const S* a, size_t idx, int i, double rho0) {
    if constexpr (PREC == PSCLBM_FP64) {
      return a[idx];
    } else if constexpr (PREC == PSCLBM_FP32) {
      return Lattice<Q>::w(i) * rho0 + static_cast<double>(a[idx]);
    } else {
      return Lattice<Q>::w(i) * rho0 +
             static_cast<double>(static_cast<float>(a[idx])) * Lattice<Q>::w(i);
    }
  }
  __device__ static void from_f64(S* a, size_t idx, int i, double f, double rho0) {
    const double g = f - Lattice<Q>::w(i) * rho0;
    if constexpr (PREC == PSCLBM_FP64) {
      a[idx] = f;
    } else if constexpr (PREC == PSCLBM_FP32) {
      a[idx] = static_cast<float>(g);
    } else {
      a[idx] = static_cast<_Float16>(static_cast<float>(g / Lattice<Q>::w(i)));
    }
  }
};

// ---------------------------------------------------------------------------
// Neighbour addressing with periodic wrap; returns false when the link leaves
// through a non-periodic face (and accumulates that face's wall velocity).
// ---------------------------------------------------------------------------
struct Cell {
  int x, y, z;
  long long n;
};

__device__ inline bool neighbour(const Geom& g, const Cell& c, int dx, int dy, int dz,
                                 long long& m, double* uw) {
  int p[3] = {c.x + dx, c.y + dy, c.z + dz};
  const int L[3] = {g.nx, g.ny, g.nz};
  bool inside = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (p[a] < 0 || p[a] >= L[a]) {
      if (g.periodic[a]) {
        p[a] += p[a] < 0 ? L[a] : -L[a];
      } else {
        inside = false;
        if (uw) {
          const int face = 2 * a + (p[a] < 0 ? 0 : 1);
          if (g.face[face] == PSCLBM_MOVING_WALL) {
            uw[0] += g.face_u[face][0];
            uw[1] += g.face_u[face][1];
            uw[2] += g.face_u[face][2];
          }
        }
      }
    }
  }
  m = p[0] + (long long)g.nx * (p[1] + (long long)g.ny * p[2]);
  return inside;
}

// Canonical population i of cell c at streaming parity par: its storage index.
template <int Q>
__device__ inline size_t canonical_index(const Geom& g, const Cell& c, int i, int par) {
  if (par == 0) return (size_t)i * g.N + c.n;
  long long m;
  if (neighbour(g, c, -Lattice<Q>::ex(i), -Lattice<Q>::ey(i), -Lattice<Q>::ez(i), m, nullptr))
    return (size_t)Lattice<Q>::opp(i) * g.N + m;
  return (size_t)i * g.N + c.n;
}

__device__ inline Cell cell_of(const Geom& g, long long n) {
  Cell c;
  c.n = n;
  c.x = (int)(n % g.nx);
  long long r = n / g.nx;
  c.y = (int)(r % g.ny);
  c.z = (int)(r / g.ny);
  return c;
}

// ---------------------------------------------------------------------------
// The fused collide-stream step.
// ---------------------------------------------------------------------------
// Waves per SIMD of each form, the register budget of the tiles (which the
// contact workgroups' code must fit as well), each as measured fastest: 2D
// FP32 / FP16 8 (their slot fractions held in FP32, so that eight
// workgroups' LDS fits a CU), walled 3D FP32 / FP16 7, periodic 3D FP32 /
// FP16 6 (the per-cell moments keep their registers lower), 2D FP64 5, 3D
// FP64 4.  The reduced 3D forms are bound by instruction issue, and more
// waves hide more of the loads' and the tile list's latency under it, up to
// the point where spills cost more.
template <int Q, int PREC, bool WALLS>
constexpr int step_waves() {
  if (PREC == PSCLBM_FP64) return Q == 9 ? 5 : 4;
  if (Q == 9) return 8;
  return WALLS ? 7 : 6;
}

// NT (even steps only): the lattice is streamed with non-temporal loads and
// stores, each line being read and written by one wave.
template <int Q, int PREC, int PAR, bool WALLS, bool NT = false>
__global__ void __launch_bounds__(BLOCK)
    __attribute__((amdgpu_waves_per_eu(step_waves<Q, PREC, WALLS>())))
    k_step(const StepArgs a) {
  static_assert(!NT || PAR == 0, "non-temporal streaming in the even steps only");
  using L = Lattice<Q>;
  using C = typename Form<PREC>::C;
  using S = typename Form<PREC>::S;
  using ST = Store<PREC, Q>;
  constexpr int D = L::D;
  // slot fractions held in FP32 by the FP32 arithmetic forms
  using E = typename std::conditional<PREC == PSCLBM_FP64, double, float>::type;
  constexpr bool SC = scaled_form<PREC>();
  extern __shared__ double smem_d[];
  __shared__ SlotLdsT<E> slot_lds;
  if ((int)blockIdx.x < a.dem_blocks) {
    // contact workgroup of the coupled step: one wave per particle gathers
    // its DEM contact force from the binning of the step's start
    const int i = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (BLOCK / 64) + threadIdx.x / 64));
    if (i < a.dem.n) {
      const int lane = (int)(threadIdx.x & 63);
      double xs[3], us[3], fs[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        xs[k] = a.px[3 * i + k];
        us[k] = a.pu[3 * i + k];
      }
      dem_contact_wave(a.dem, i, lane, xs, us, a.pr[i], fs);
      if (lane == 0)
#pragma unroll
        for (int k = 0; k < 3; ++k) a.fc[3 * i + k] = fs[k];
    }
    return;
  }
  S* __restrict__ A = static_cast<S*>(a.f);
  // the tiles: workgroups dem_blocks.. (a multiple of 8, so that the XCD
  // round robin of the tile workgroups is that of their own index)
  const int nb = (int)gridDim.x - a.dem_blocks;
  const int bid = (int)blockIdx.x - a.dem_blocks;
  const int tile = tile_of(a.g, bid, nb);

  // particle list of the tile (LDS) and its force accumulators
  LdsEntry* lds = reinterpret_cast<LdsEntry*>(smem_d);
  double* acc = reinterpret_cast<double*>(lds + a.cap);
  const int cnt = load_tile_list(a.tile_count, a.tile_list, a.cap, a.snap, tile, lds, acc, a.np);

  const Dims d = dims_of(a.g);
  // the wave's 64-cell row segment; y and z are uniform over the wave (scalar)
  int x0, y, z;
  wave_segment(a.g, tile, x0, y, z);
  const int x = x0 + (int)(threadIdx.x & 63);
  const bool active = x < d.nx && y < d.ny && z < d.nz;
  const unsigned n = (unsigned)x + d.sy * (unsigned)y + d.sz * (unsigned)z;
  const unsigned N = (unsigned)a.g.N;
  const double rho0 = a.g.rho0;
  double mass_dev = 0.0;
  // the wave's cells and all their neighbours inside the lattice (no face
  // within one cell of the segment): every link is the plain offset, with no
  // wrap and no wall (uniform over the wave).  Taken by the odd steps of the
  // FP32 form and of the walled FP16 one, whose pulled loads and pushed
  // stores otherwise resolve 2 x 18 links (the walled 384x192x192 odd step
  // 503 -> 449 us in FP32, 496 -> 436 us in FP16); in the other forms the
  // second copy of the loops measured neutral to 2 % slower.
  constexpr bool INNER_PATH =
      PAR == 1 && (PREC == PSCLBM_FP32 || (PREC == PSCLBM_FP32_FP16STORE && WALLS));
  const bool inner = INNER_PATH &&
                     __builtin_amdgcn_readfirstlane(
                         (int)(x0 >= 1 && x0 + SEG <= d.nx - 1 && y >= 1 && y <= d.ny - 2 &&
                               (D == 2 || (z >= 1 && z <= d.nz - 2)))) != 0;

  // ---- solid fractions of the covering particles (Table 1), whole wave; in
  // 3D after the loads of f are issued, so that their latency overlaps the
  // slot search (in 2D the registers this holds cost more than it saves) ----
  SlotsT<E> s;
  s.n = 0;
  if constexpr (Q == 9) {
    if (cnt > 0) collect_slots<D>(a.g, x0, y, z, active, lds, cnt, a.h, s, a.err, slot_lds);
  }

  C g[Q];
  C rho = (C)1, ux = 0, uy = 0, uz = 0, uu = 0;
  C Bn_cell = 0;
  // uniform parameters in the compute type (the FP32 copies are rounded on
  // the host, to the values a conversion here would give)
  auto uni = [](double v, float vf) -> C {
    if constexpr (std::is_same<C, double>::value) { (void)vf; return v; }
    else { (void)v; return vf; }
  };
  const C F0 = uni(a.force[0], a.force_f[0]), F1 = uni(a.force[1], a.force_f[1]),
          F2 = uni(a.force[2], a.force_f[2]);
  const C rho0c = uni(a.g.rho0, a.rho0_f), inv_rho0 = uni(a.inv_rho0, a.inv_rho0_f);
  const double tm = a.tau - 0.5;
  E bscale = 1;  // B_s / eps_{n,s} of the cell (Eq. 13), formed with the weights
  if (active) {
    // ---- load f as deviations g_i = f_i - w_i rho0 ----
    bool loaded = false;
    if constexpr (INNER_PATH) {
      if (inner) {  // plain offsets
#pragma unroll
        for (int i = 0; i < Q; ++i)
          g[i] = ST::ld(A + (size_t)L::opp(i) * N, n - link_offset<L>(d, i), i, rho0);
        loaded = true;
      }
    }
    if (!loaded) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        if constexpr (PAR == 2) {
          g[i] = ST::ld(dir_ptr(const_cast<S*>(static_cast<const S*>(a.src)), i, N), n, i, rho0);
        } else if constexpr (PAR == 0) {
          g[i] = ST::template ld<NT>(dir_ptr(A, i, N), n, i, rho0);
        } else {
          unsigned m = n;
          if (!link<WALLS>(d, x, y, z, -L::ex(i), -L::ey(i), -L::ez(i), n, m))
            g[i] = ST::ld(A + (size_t)L::opp(i) * N, m, i, rho0);
          else  // reflected at a wall during the previous (even) step
            g[i] = ST::ld(A + (size_t)i * N, n, i, rho0);
        }
      }
    }
  }
  if constexpr (Q == 19) {
    if (cnt > 0) collect_slots<D>(a.g, x0, y, z, active, lds, cnt, a.h, s, a.err, slot_lds);
  }
  // the slots' list entries, two to a register (entries < 2^16; the list
  // capacity is at most 512): registers held through the collision
  const unsigned e01 = (unsigned)s.e[0] | ((unsigned)s.e[1] << 16);
  const unsigned e23 = (unsigned)s.e[2] | ((unsigned)s.e[3] << 16);
  auto slot_e = [&](int k) {
    return (int)(((k < 2 ? e01 : e23) >> (16 * (k & 1))) & 0xffffu);
  };
  static_assert(KSLOTS == 4, "entries packed for four slots");

  // ---- the covering particles, slot by slot ----
  // the row's y and z as FP64, converted from their scalar registers at each
  // use: an empty asm makes each use opaque, so the compiler does not hold
  // (or spill) one converted copy across the slots
  auto row_coord = [](int v) {
    asm volatile("" : "+s"(v));
    return (double)v;
  };
  constexpr int NV = D == 3 ? 6 : 3;
  // particle s of slot k at this cell: its share B_s, the weight of its
  // momentum exchange (Eq. 14 weighs it by B_s, Eq. 11 by the cell's B_n),
  // u_s - u and u_s + u with u_s the rigid-body velocity at the cell centre,
  // and the cell centre's offset from the particle centre
  struct SlotKin {
    C Bs, Bm, dv[3], sv[3], r[3];
  };
  auto slot_kin = [&](int k) {
    SlotKin t;
    t.Bs = a.original ? (C)(s.eps[k] * tm / ((1.0 - s.eps[k]) + tm)) : (C)(s.eps[k] * bscale);
    t.Bm = a.original ? Bn_cell : t.Bs;
    const LdsEntry& P = lds[slot_e(k)];
    // u_s = U + Omega x r in the arithmetic precision: the arm from its FP64
    // nearest image, or in the FP32 forms from the centre's FP32 pair
    C cx, cy, cz;
    if constexpr (PREC == PSCLBM_FP64) {
      cx = min_image((double)x - P.x, d.px, d.nx);
      cy = min_image(row_coord(y) - P.y, d.py, d.ny);
      cz = D == 3 ? min_image(row_coord(z) - P.z, d.pz, d.nz) : 0.0;
    } else {
      cx = min_image_f((float)x - P.xh[0], d.px, d.nx) - P.xl[0];
      cy = min_image_f((float)y - P.xh[1], d.py, d.ny) - P.xl[1];
      cz = D == 3 ? min_image_f((float)z - P.xh[2], d.pz, d.nz) - P.xl[2] : 0.0f;
    }
    C U[3], W[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if constexpr (PREC == PSCLBM_FP64) {
        U[c] = P.u[c];
        W[c] = P.w[c];
      } else {
        U[c] = P.uf[c];
        W[c] = P.wf[c];
      }
    }
    const C usx = U[0] + W[1] * cz - W[2] * cy;
    const C usy = U[1] + W[2] * cx - W[0] * cz;
    const C usz = D == 3 ? U[2] + W[0] * cy - W[1] * cx : (C)0;
    t.dv[0] = usx - ux;
    t.dv[1] = usy - uy;
    t.dv[2] = usz - uz;
    t.sv[0] = usx + ux;
    t.sv[1] = usy + uy;
    t.sv[2] = usz + uz;
    t.r[0] = cx;
    t.r[1] = cy;
    t.r[2] = cz;
    return t;
  };
  // the negated momentum exchange of Eq. 14, m_s = B [rho (u_s - u) + F]:
  // force, then torque about the particle centre
  auto exchange = [&](const SlotKin& t, C (&mv)[NV]) {
    const C mx = t.Bm * (rho * t.dv[0] + F0);
    const C my = t.Bm * (rho * t.dv[1] + F1);
    mv[0] = -mx;
    mv[1] = -my;
    if constexpr (D == 3) {
      const C mz = t.Bm * (rho * t.dv[2] + F2);
      mv[2] = -mz;
      mv[3] = -(t.r[1] * mz - t.r[2] * my);
      mv[4] = -(t.r[2] * mx - t.r[0] * mz);
      mv[5] = -(t.r[0] * my - t.r[1] * mx);
    } else {
      mv[2] = -(t.r[0] * my - t.r[1] * mx);
    }
  };
  // added to the list entry's FP64 accumulators in LDS
  auto accumulate = [&](int e, const C (&mv)[NV]) {
    double* ac = acc + 6 * e;
    atomicAdd(ac + 0, (double)mv[0]);
    atomicAdd(ac + 1, (double)mv[1]);
    if constexpr (D == 3) {
      atomicAdd(ac + 2, (double)mv[2]);
      atomicAdd(ac + 3, (double)mv[3]);
      atomicAdd(ac + 4, (double)mv[4]);
      atomicAdd(ac + 5, (double)mv[5]);
    } else {
      atomicAdd(ac + 5, (double)mv[2]);
    }
  };
  // periodic 3D reduced-precision forms: the particles' equilibrium difference
  // enters the collision through ten per-cell moments (one pass over the
  // directions); the others add it slot by slot after the collision (with
  // walls, the moments' registers cost spills of loaded populations)
  constexpr bool FOLD = D == 3 && PREC != PSCLBM_FP64 && !WALLS;
  // no body force: the Guo terms vanish (uniform over the launch)
  const bool forced = __builtin_amdgcn_readfirstlane(
                          (int)(a.force[0] != 0.0 || a.force[1] != 0.0 || a.force[2] != 0.0)) != 0;

  if (active) {
    // ---- inlet / outlet layers: reset to an equilibrium before collision ----
    if (a.open_mask) {
      bool reset = false;
      double ub0 = 0.0, ub1 = 0.0, ub2 = 0.0;
      // x-face outlets: the velocity of the interior neighbour at this time
      // level, from the neighbour's lane of this wave
      double wu0 = 0.0, wu1 = 0.0, wu2 = 0.0;
      if (a.outlet_wave) {
        C r_, j0, j1, j2;
        cell_moments<Q, SC>(g, r_, j0, j1, j2);
        const int lane = (int)(threadIdx.x & 63);
        int src = lane;
        if ((a.outlet_wave & 1u) && x == 0) src = lane + 1;
        if ((a.outlet_wave & 2u) && x == d.nx - 1) src = lane - 1;
        r_ = __shfl(r_, src);
        j0 = __shfl(j0, src);
        j1 = __shfl(j1, src);
        j2 = __shfl(j2, src);
        const C ir = inv_density(rho0c + r_);
        const C qr = r_ * ir, ir0 = inv_rho0;
        wu0 = (double)eq5_velocity(j0, (C)0.5 * F0, qr, ir, ir0);
        wu1 = (double)eq5_velocity(j1, (C)0.5 * F1, qr, ir, ir0);
        wu2 = (double)eq5_velocity(j2, (C)0.5 * F2, qr, ir, ir0);
      }
#pragma unroll
      for (int f = 0; f < 6; ++f) {  // outlets first, an inlet wins on a corner
        const bool on = f == 0 ? x == 0 : f == 1 ? x == d.nx - 1 : f == 2 ? y == 0
                      : f == 3 ? y == d.ny - 1 : f == 4 ? z == 0 : z == d.nz - 1;
        if (((a.outlet_mask >> f) & 1u) && on) {
          if ((a.outlet_wave >> f) & 1u) {
            ub0 = wu0;
            ub1 = wu1;
            ub2 = wu2;
          } else {
            const unsigned k = f < 2 ? (unsigned)y + (unsigned)d.ny * z
                                     : (f < 4 ? (unsigned)x + (unsigned)d.nx * z
                                              : (unsigned)x + (unsigned)d.nx * y);
            const double* o = a.outlet_u + ((size_t)f * a.face_stride + k) * 3;
            ub0 = o[0];
            ub1 = o[1];
            ub2 = o[2];
          }
          reset = true;
        }
      }
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        const bool on = f == 0 ? x == 0 : f == 1 ? x == d.nx - 1 : f == 2 ? y == 0
                      : f == 3 ? y == d.ny - 1 : f == 4 ? z == 0 : z == d.nz - 1;
        if (((a.inlet_mask >> f) & 1u) && on) {
          ub0 = a.g.face_u[f][0];
          ub1 = a.g.face_u[f][1];
          ub2 = a.g.face_u[f][2];
          reset = true;
        }
      }
      if (reset) {
        const C u0 = (C)ub0, u1 = (C)ub1, u2 = (C)ub2;
        const C uq = u0 * u0 + u1 * u1 + u2 * u2;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const C eu = edot(L::ex(i), L::ey(i), L::ez(i), u0, u1, u2);
          g[i] = wq<Q, SC>(i, (C)rho0 * ((C)3 * eu + (C)4.5 * eu * eu - (C)1.5 * uq));
        }
      }
    }

    // ---- moments with the half-force shift (Eq. 5) ----
    C drho, jx, jy, jz;
    cell_moments<Q, SC>(g, drho, jx, jy, jz);
    rho = rho0c + drho;
    const C inv_rho = inv_density(rho);
    const C q_rho = drho * inv_rho;
    if (forced) {
      ux = eq5_velocity(jx, (C)0.5 * F0, q_rho, inv_rho, inv_rho0);
      uy = eq5_velocity(jy, (C)0.5 * F1, q_rho, inv_rho, inv_rho0);
      uz = eq5_velocity(jz, (C)0.5 * F2, q_rho, inv_rho, inv_rho0);
    } else {
      ux = eq5_velocity_unforced(jx, q_rho, inv_rho, inv_rho0);
      uy = eq5_velocity_unforced(jy, q_rho, inv_rho, inv_rho0);
      uz = eq5_velocity_unforced(jz, q_rho, inv_rho, inv_rho0);
    }
    uu = ux * ux + uy * uy + uz * uz;
    const C omega = uni(a.omega, a.omega_f);
    const C kguo = (C)1 - (C)0.5 * omega;
    const C uF = ux * F0 + uy * F1 + uz * F2;

    // Weights (Eq. 13 with the cell total clamped at one, Table 1): B_n from
    // the clamped cell total, each particle's share B_s per slot.  The
    // original weighting (Eq. 9) takes each particle's B_s from its own
    // fraction and B_n as their sum.
    // In the precision the fractions are held in: FP64, or FP32 with the
    // hardware reciprocal (1 ulp) for the FP32 arithmetic forms; the
    // denominators are at least tau - 1/2 > 0.
    auto recip = [](E v) -> E {
      if constexpr (PREC == PSCLBM_FP64) return 1.0 / v;
      else return __builtin_amdgcn_rcpf(v);
    };
    E S_ = 0;
#pragma unroll
    for (int k = 0; k < KSLOTS; ++k)
      if (k < s.n) S_ += s.eps[k];
    const E tme = uni(tm, a.tm_f);  // E is the compute type
    const E en = S_ < (E)1 ? S_ : (E)1;
    const E den = ((E)1 - en) + tme;
    E inv_den = 1;
    if (s.n > 0) inv_den = recip(den);
    // share of each particle: Eq. 13 when the fractions sum to at most one,
    // else eps_{n,s} / sum (the clamped total has B_n = 1)
    bscale = tme * inv_den;
    if (S_ > (E)1) bscale = recip(S_);
    E Bn_e = s.n > 0 ? en * tme * inv_den : (E)0;
    // a covered cell (en = 1) has B_n = 1 exactly, which the reciprocal's
    // last bit must not undo (no BGK part may act there)
    if constexpr (PREC != PSCLBM_FP64)
      if (en >= (E)1) Bn_e = (E)1;
    if (a.original) {
      double Bn_d = 0.0;
#pragma unroll
      for (int k = 0; k < KSLOTS; ++k)
        if (k < s.n) Bn_d += s.eps[k] * tm / ((1.0 - s.eps[k]) + tm);
      Bn_e = (E)Bn_d;
    }
    const C Bn = (C)Bn_e;
    Bn_cell = Bn;
    const C omB = (C)1 - Bn;
    const C relax = omB * omega;

    if constexpr (FOLD) {
      // ---- the slots: the moments A = sum_s B_s (u_s - u) and the symmetric
      // M = sum_s B_s (u_s u_s - u u) (diagonal in mD, off-diagonal doubled
      // in mH, formed as B_s [(u_s - u)(u_s + u)^T + transpose] / 2), and the
      // momentum exchange ----
      C mA[3] = {0, 0, 0}, mD[3] = {0, 0, 0}, mH[3] = {0, 0, 0};
      if (s.n > 0) {
#pragma unroll
        for (int k = 0; k < KSLOTS; ++k) {
          if (k >= s.n) continue;
          const SlotKin t = slot_kin(k);
          C b[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            b[c] = t.Bs * t.dv[c];
            mA[c] += b[c];
            mD[c] += b[c] * t.sv[c];
          }
          mH[0] += b[0] * t.sv[1] + b[1] * t.sv[0];
          mH[1] += b[0] * t.sv[2] + b[2] * t.sv[0];
          mH[2] += b[1] * t.sv[2] + b[2] * t.sv[1];
          if (a.facc) {
            C mv[NV];
            exchange(t, mv);
            accumulate(slot_e(k), mv);
          }
        }
      }
      // ---- one pass over the directions: BGK + Guo weighted by 1 - B_n, the
      // bounce-back of the non-equilibrium part, B_n (fneq_{-i} - fneq_i), and
      // the particles' sum_s B_s [f^eq_i(rho, u_s) - f^eq_i(rho, u)], which is
      // w_i rho [3 e_i.A + 4.5 e_i.M.e_i - 1.5 tr M] (Eqs. 2-4, 10-12) ----
      const C r3 = (C)3 * rho, r45 = (C)4.5 * rho;
      const C pA[3] = {r3 * mA[0], r3 * mA[1], r3 * mA[2]};
      const C pD[3] = {r45 * mD[0], r45 * mD[1], r45 * mD[2]};
      const C pH[3] = {r45 * mH[0], r45 * mH[1], r45 * mH[2]};
      const C p0 = (C)-1.5 * rho * (mD[0] + mD[1] + mD[2]);
      auto collide = [&](auto guo) {
        constexpr bool GUO = decltype(guo)::value;
        const C gk = omB * kguo;
        // g_i - relax fneq_i + B_n (fneq_-i - fneq_i) as g_i - (relax + B_n)
        // fneq_i + B_n fneq_-i: the non-equilibrium parts stay explicit, so an
        // equilibrium is kept exactly (no rounding of 1 - relax - B_n enters)
        const C rB = relax + Bn;
        {
          C x0 = p0;
          if constexpr (GUO) x0 -= gk * (C)3 * uF;
          const C fneq = g[0] - wq<Q, SC>(0, drho - rho * (C)1.5 * uu);
          g[0] = g[0] - relax * fneq + wq<Q, SC>(0, x0);
        }
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          const int o = L::opp(i);
          if (o < i) continue;
          const int ex = L::ex(i), ey = L::ey(i), ez = L::ez(i);
          const C eu = edot(ex, ey, ez, ux, uy, uz);
          const C sym = drho + rho * ((C)4.5 * eu * eu - (C)1.5 * uu);
          const C fn_i = g[i] - wq<Q, SC>(i, sym + rho * (C)3 * eu);
          const C fn_o = g[o] - wq<Q, SC>(i, sym - rho * (C)3 * eu);
          // the even and odd parts under e -> -e of the particles' term and
          // of the Guo term (Eq. 4)
          C ps = p0;
          eacc(ex * ex, ps, pD[0]);
          eacc(ey * ey, ps, pD[1]);
          eacc(ez * ez, ps, pD[2]);
          eacc(ex * ey, ps, pH[0]);
          eacc(ex * ez, ps, pH[1]);
          eacc(ey * ez, ps, pH[2]);
          C pa = edot(ex, ey, ez, pA[0], pA[1], pA[2]);
          if constexpr (GUO) {
            const C eF = edot(ex, ey, ez, F0, F1, F2);
            ps += gk * ((C)9 * eu * eF - (C)3 * uF);
            pa += gk * ((C)3 * eF);
          }
          g[i] = g[i] - rB * fn_i + Bn * fn_o + wq<Q, SC>(i, ps + pa);
          g[o] = g[o] - rB * fn_o + Bn * fn_i + wq<Q, SC>(i, ps - pa);
        }
      };
      if (forced)
        collide(std::true_type{});
      else
        collide(std::false_type{});
    } else {
      // ---- pass 1: BGK + Guo weighted by (1 - B_n), plus the bounce-back of
      // the non-equilibrium part, B_n (fneq_{-i} - fneq_i); one opposite pair
      // at a time (Eqs. 2-4, 10, 12), the relaxation and the bounce-back
      // applied as in the folded collision above ----
      const C rB = relax + Bn;
      {
        const C wi = SC ? (C)1 : (C)L::w(0);
        const C fneq = g[0] - wq<Q, SC>(0, drho - rho * (C)1.5 * uu);
        g[0] = g[0] - relax * fneq - omB * kguo * wi * (C)3 * uF;
      }
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const int o = L::opp(i);
        if (o < i) continue;
        const C wi = SC ? (C)1 : (C)L::w(i);
        const C eu = edot(L::ex(i), L::ey(i), L::ez(i), ux, uy, uz);
        const C eF = edot(L::ex(i), L::ey(i), L::ez(i), F0, F1, F2);
        const C sym = drho + rho * ((C)4.5 * eu * eu - (C)1.5 * uu);
        const C fn_i = g[i] - wq<Q, SC>(i, sym + rho * (C)3 * eu);
        const C fn_o = g[o] - wq<Q, SC>(i, sym - rho * (C)3 * eu);
        // Guo term (Eq. 4): even and odd parts under e -> -e
        const C Fsym = kguo * wi * ((C)9 * eu * eF - (C)3 * uF);
        const C Fant = kguo * wi * ((C)3 * eF);
        g[i] = g[i] - rB * fn_i + Bn * fn_o + omB * (Fsym + Fant);
        g[o] = g[o] - rB * fn_o + Bn * fn_i + omB * (Fsym - Fant);
      }
    }
  }

  // ---- pass 2 (covered cells of the other forms): sum_s B_s [f^eq_i(rho,
  // u_s) - f^eq_i(rho, u)] and the momentum exchange ----
  if constexpr (!FOLD) {
    // slot k of this cell: the equilibrium difference into g and, unless the
    // step accumulates no force (the ring step), the negated exchange into mv
    auto slot_update = [&](int k, C (&mv)[NV]) {
      const SlotKin t = slot_kin(k);
      const C du2 = t.dv[0] * t.sv[0] + t.dv[1] * t.sv[1] + t.dv[2] * t.sv[2];  // |u_s|^2 - |u|^2
      const C rB = rho * t.Bs;
      g[0] -= wq<Q, SC>(0, rB * (C)1.5 * du2);
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const int o = L::opp(i);
        if (o < i) continue;
        const C de = edot(L::ex(i), L::ey(i), L::ez(i), t.dv[0], t.dv[1], t.dv[2]);
        const C se = edot(L::ex(i), L::ey(i), L::ez(i), t.sv[0], t.sv[1], t.sv[2]);
        // 4.5 [(e.u_s)^2 - (e.u)^2] - 1.5 (|u_s|^2 - |u|^2), and 3 e.(u_s - u)
        const C ds_s = (C)4.5 * de * se - (C)1.5 * du2;
        const C ds_a = (C)3 * de;
        g[i] += wq<Q, SC>(i, rB * (ds_s + ds_a));
        g[o] += wq<Q, SC>(i, rB * (ds_s - ds_a));
      }
      if (a.facc) exchange(t, mv);
    };
    if constexpr (PREC == PSCLBM_FP64 || D == 3) {
      // every covered lane adds its own exchange (the LDS unit serialises
      // lanes of one entry; the block sums below would cost FP64 registers)
      if (s.n > 0) {
#pragma unroll
        for (int k = 0; k < KSLOTS; ++k) {
          if (k >= s.n) continue;
          C mv[NV];
          slot_update(k, mv);
          if (a.facc) accumulate(slot_e(k), mv);
        }
      }
    } else {
      // slot by slot over the wave: the exchange is first summed over
      // aligned blocks of up to 8 lanes whose slot holds the same entry, and
      // only each block's leader adds it to LDS
      const int lane = (int)(threadIdx.x & 63);
#pragma unroll
      for (int k = 0; k < KSLOTS; ++k) {
        const bool has = k < s.n;
        if (!__any(has)) break;  // uniform over the wave
        C mv[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) mv[j] = 0;
        if (has) slot_update(k, mv);
        if (a.facc) {
          bool lead;
          const unsigned mf = merge_flags(has ? slot_e(k) : -1, lane, lead);
#pragma unroll
          for (int j = 0; j < NV; ++j) mv[j] = merge_sum(mv[j], mf);
          if (lead) accumulate(slot_e(k), mv);
        }
      }
    }
  }

  if (active) {
    // ---- stream (Eq. 1) with halfway bounce-back (Eq. 6) ----
    // the cell index formed again from x (an empty asm keeps the compiler from
    // reusing, and so holding or spilling, the one the loads used)
    unsigned xo = (unsigned)x;
    asm volatile("" : "+v"(xo));
    const unsigned no = xo + d.sy * (unsigned)y + d.sz * (unsigned)z;
    double cell_dev = 0.0;  // FP64 sum of the stored deviations, in every form
    bool stored = false;
    if constexpr (INNER_PATH) {
      if (inner) {  // plain offsets: every population to its neighbour
#pragma unroll
        for (int i = 0; i < Q; ++i)
          cell_dev += ST::st(A + (size_t)i * N, no + link_offset<L>(d, i), i, g[i], rho0);
        stored = true;
      }
    }
    if (!stored) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      unsigned m = no;
      // the even step stores into the own cell: its links matter only for a
      // moving wall's term
      const unsigned out =
          (i == 0 || (PAR == 0 && !a.moving_mask))
              ? 0u
              : link<WALLS>(d, x, y, z, L::ex(i), L::ey(i), L::ez(i), no, m);
      C v = g[i];
      if (out) {
        const unsigned mw = out & a.moving_mask;
        if (mw) {  // moving wall: -2 w_i rho (e_i . u_w) / c_s^2
          double uw0 = 0.0, uw1 = 0.0, uw2 = 0.0;
#pragma unroll
          for (int f = 0; f < 6; ++f)
            if ((mw >> f) & 1u) {
              uw0 += a.g.face_u[f][0];
              uw1 += a.g.face_u[f][1];
              uw2 += a.g.face_u[f][2];
            }
          const double eu = edot(L::ex(i), L::ey(i), L::ez(i), uw0, uw1, uw2);
          v -= (C)(6.0 * (SC ? 1.0 : L::w(i)) * eu) * rho;
        }
      }
      if (PAR == 0)  // own cell, opposite slot
        cell_dev += ST::template st<NT>(dir_ptr(A, L::opp(i), N), no, i, v, rho0);
      else if (out)  // reflected into the own cell's opposite slot
        cell_dev += ST::st(A + (size_t)L::opp(i) * N, no, i, v, rho0);
      else                  // neighbour cell, same slot
        cell_dev += ST::st(A + (size_t)i * N, m, i, v, rho0);
    }
    }
    mass_dev = cell_dev;
  }

  // ---- per-workgroup FP64 mass partial (sum of the stored deviations) ----
  __shared__ double wsum[BLOCK / 64];
  if (a.mass_part) {
    mass_dev = wave_sum(mass_dev);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = mass_dev;
  }
  __syncthreads();
  if (a.mass_part && threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < BLOCK / 64; ++k) t += wsum[k];
    a.mass_part[bid] = t;
  }

  // ---- flush the tile's force / torque partials (FP64), one (entry,
  // component) pair per thread so that a tile's atomics are issued together
  // rather than six in turn by each entry's thread (256^3 FP32 step 576 ->
  // 541 us); the barrier of the mass reduction above orders the LDS
  // accumulation before this read ----
  if (cnt > 0 && a.facc) {
    for (int t = threadIdx.x; t < 6 * cnt; t += BLOCK) {
      const int e = t / 6, k = t - 6 * e;
      const double v = acc[t];
      if (v != 0.0) atomicAdd(a.facc + 6 * (size_t)lds[e].id + k, v);
    }
  }
  // ---- clear the other force buffer for the next step ----
  if (a.np > 0 && a.fzero) {
    const unsigned tot = 6u * (unsigned)a.np;
    for (unsigned k = (unsigned)bid * BLOCK + threadIdx.x; k < tot; k += (unsigned)nb * BLOCK)
      a.fzero[k] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Outlet layers: velocity (Eq. 5) of the interior neighbour of every outlet
// cell at the current time level, read before the step kernel runs.
// ---------------------------------------------------------------------------
template <int Q, int PREC>
__global__ void k_outlet_velocity(Geom g, const void* f, int par, double fx, double fy,
                                  double fz, double* out, long long stride, unsigned faces) {
  using L = Lattice<Q>;
  using ST = Store<PREC, Q>;
  using S = typename Form<PREC>::S;
  const int face = blockIdx.y;
  if (!((faces >> face) & 1u)) return;
  const int ax = face / 2;
  const int u1 = ax == 0 ? 1 : 0, u2 = ax == 2 ? 1 : 2;
  const int Ld[3] = {g.nx, g.ny, g.nz};
  const long long cells = (long long)Ld[u1] * Ld[u2];
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < cells;
       k += (long long)gridDim.x * blockDim.x) {
    int p[3];
    p[u1] = (int)(k % Ld[u1]);
    p[u2] = (int)(k / Ld[u1]);
    p[ax] = (face % 2 == 0) ? 1 : Ld[ax] - 2;
    Cell c;
    c.x = p[0];
    c.y = p[1];
    c.z = p[2];
    c.n = c.x + (long long)g.nx * (c.y + (long long)g.ny * c.z);
    double rho = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
      const double fi = ST::to_f64(static_cast<const S*>(f), canonical_index<Q>(g, c, i, par), i,
                                   g.rho0);
      rho += fi;
      j[0] += L::ex(i) * fi;
      j[1] += L::ey(i) * fi;
      j[2] += L::ez(i) * fi;
    }
    double* o = out + ((size_t)face * stride + k) * 3;
    o[0] = (j[0] + 0.5 * fx) / rho;
    o[1] = (j[1] + 0.5 * fy) / rho;
    o[2] = (j[2] + 0.5 * fz) / rho;
  }
}

// ---------------------------------------------------------------------------
// State I/O
// ---------------------------------------------------------------------------
template <int Q, int PREC>
__global__ void k_set_equilibrium(Geom g, void* f, const double* rho, const double* u) {
  using L = Lattice<Q>;
  using S = typename Form<PREC>::S;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < g.N;
       n += (long long)gridDim.x * blockDim.x) {
    const double r = rho ? rho[n] : g.rho0;
    double ub[3] = {0, 0, 0};
    if (u) {
      ub[0] = u[3 * n];
      ub[1] = u[3 * n + 1];
      ub[2] = u[3 * n + 2];
    }
    const double uu = ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2];
    for (int i = 0; i < Q; ++i) {
      const double eu = L::ex(i) * ub[0] + L::ey(i) * ub[1] + L::ez(i) * ub[2];
      const double fe = r * L::w(i) * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
      Store<PREC, Q>::from_f64(static_cast<S*>(f), (size_t)i * g.N + n, i, fe, g.rho0);
    }
  }
}

template <int Q, int PREC>
__global__ void k_set_f(Geom g, void* f, const double* src) {
  using S = typename Form<PREC>::S;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < g.N;
       n += (long long)gridDim.x * blockDim.x)
    for (int i = 0; i < Q; ++i)
      Store<PREC, Q>::from_f64(static_cast<S*>(f), (size_t)i * g.N + n, i,
                               src[(size_t)i * g.N + n], g.rho0);
}

template <int Q, int PREC>
__global__ void k_get_f(Geom g, const void* f, int par, double* dst, double* rho, double* u,
                        double fx, double fy, double fz) {
  using L = Lattice<Q>;
  using S = typename Form<PREC>::S;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < g.N;
       n += (long long)gridDim.x * blockDim.x) {
    const Cell c = cell_of(g, n);
    double m = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
      const double fi = Store<PREC, Q>::to_f64(static_cast<const S*>(f),
                                               canonical_index<Q>(g, c, i, par), i, g.rho0);
      if (dst) dst[(size_t)i * g.N + n] = fi;
      m += fi;
      j[0] += L::ex(i) * fi;
      j[1] += L::ey(i) * fi;
      j[2] += L::ez(i) * fi;
    }
    if (rho) rho[n] = m;
    if (u) {
      u[3 * n] = (j[0] + 0.5 * fx) / m;
      u[3 * n + 1] = (j[1] + 0.5 * fy) / m;
      u[3 * n + 2] = (j[2] + 0.5 * fz) / m;
    }
  }
}

// Mass of the current state, per workgroup (sum of stored deviations).
template <int Q, int PREC>
__global__ void __launch_bounds__(256) k_mass_direct(Geom g, const void* f, double* part) {
  using S = typename Form<PREC>::S;
  double t = 0.0;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < g.N;
       n += (long long)gridDim.x * blockDim.x)
    for (int i = 0; i < Q; ++i)
      t += Store<PREC, Q>::to_f64(static_cast<const S*>(f), (size_t)i * g.N + n, i, g.rho0) -
           Lattice<Q>::w(i) * g.rho0;
  for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
  __shared__ double ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Deterministic two-level reduction of the per-workgroup mass partials.
__global__ void k_reduce(const double* part, int n, double* out) {
  __shared__ double s[256];
  double t = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) t += part[k];
  s[threadIdx.x] = t;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0];
}

// ---------------------------------------------------------------------------
// Rasterisation: particle snapshot, then tile binning (the candidate box X +- (r + h) of Table 1).
// ---------------------------------------------------------------------------
// One wave per particle: the particle's snapshot (with V_a of Eq. 17 / 19),
// its force / torque rows cleared in both buffers, and its entry in the list
// of every tile of its shell box (at most two runs per axis after a periodic
// wrap), the lanes striding over the tiles.  The list counts are double
// buffered: this launch fills `count` (all zero on entry) and clears `stale`,
// the counts of the previous rasterisation, for the next one.
__global__ void __launch_bounds__(256) k_rasterize(Geom g, int n, int three_d, double h,
                                                   const double* x, const double* u,
                                                   const double* w, const double* r,
                                                   PSnap* snap, int* count, int* stale,
                                                   int* tile_list, int cap, double* f0,
                                                   double* f1, unsigned* err, DemBinOut db) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (long long k = gid; k < g.ntx * (long long)g.nty * g.ntz;
       k += (long long)gridDim.x * blockDim.x)
    stale[k] = 0;
  if (db.count)
    for (long long k = gid; k < db.nbins; k += (long long)gridDim.x * blockDim.x) db.stale[k] = 0;
  const int s = (int)(gid >> 6);
  const int lane = (int)(threadIdx.x & 63);
  if (s >= n) return;  // uniform over the wave
  PSnap P;
  const bool ok = make_snap(three_d, x + 3 * s, u + 3 * s, w + 3 * s, r[s], P);
  if (lane == 0) {
    snap[s] = P;
    if (!ok) atomicOr(err, ERR_RADIUS);
    if (db.count) dem_bin_insert(db, three_d, g, s, x + 3 * s, u + 3 * s, r[s], err);
  }
  if (lane < 6) f0[6 * s + lane] = 0.0;
  else if (lane < 12) f1[6 * s + lane - 6] = 0.0;
  if (!ok) return;
  bin_tiles(g, three_d, h, P, s, lane, count, tile_list, cap, err);
}

template <int D>
__global__ void __launch_bounds__(BLOCK) k_solid_fraction(Geom g, double h, int np, int cap,
                                                        const int* tile_count, const int* tile_list,
                                                        const PSnap* snap, double* eps_total,
                                                        int* ids, double* seps, int kout,
                                                        unsigned* err) {
  extern __shared__ double smem_d[];
  __shared__ SlotLds slot_lds;
  LdsEntry* lds = reinterpret_cast<LdsEntry*>(smem_d);
  const int tile = blockIdx.x;
  const int cnt = load_tile_list(tile_count, tile_list, cap, snap, tile, lds, nullptr, np);
  int x0, y0, z0;
  wave_segment(g, tile, x0, y0, z0);
  Cell c;
  c.x = x0 + (int)(threadIdx.x & 63);
  c.y = y0;
  c.z = z0;
  const bool active = c.x < g.nx && c.y < g.ny && c.z < g.nz;
  c.n = c.x + (long long)g.nx * (c.y + (long long)g.ny * c.z);
  Slots s;
  s.n = 0;
  if (cnt > 0) collect_slots<D>(g, x0, c.y, c.z, active, lds, cnt, h, s, err, slot_lds);
  if (!active) return;
  double S_ = 0.0;
#pragma unroll
  for (int k = 0; k < KSLOTS; ++k)
    if (k < s.n) S_ += s.eps[k];
  if (eps_total) eps_total[c.n] = S_ < 1.0 ? S_ : 1.0;
  // the recorded slots (static register indices), then padding
#pragma unroll
  for (int k = 0; k < KSLOTS; ++k) {
    if (k >= kout) break;
    if (ids) ids[(size_t)c.n * kout + k] = k < s.n ? lds[s.e[k]].id : -1;
    if (seps) seps[(size_t)c.n * kout + k] = k < s.n ? s.eps[k] : 0.0;
  }
  for (int k = KSLOTS; k < kout; ++k) {
    if (ids) ids[(size_t)c.n * kout + k] = -1;
    if (seps) seps[(size_t)c.n * kout + k] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static int grid_for(long long n, int block = 256) {
  long long b = (n + block - 1) / block;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (int)b;
}

template <int Q, int PREC>
static int dispatch_step(psclbm_ctx* c, const StepArgs& a, int par, size_t lds_bytes) {
  const int nb = c->ntiles + a.dem_blocks;
  const bool walls = !(c->geom.periodic[0] && c->geom.periodic[1] && c->geom.periodic[2]);
  if (par == 2) {  // ring step: canonical FP64 in and out
    if constexpr (PREC == PSCLBM_FP64) {
      if (walls)
        k_step<Q, PREC, 2, true><<<nb, BLOCK, lds_bytes, c->stream>>>(a);
      else
        k_step<Q, PREC, 2, false><<<nb, BLOCK, lds_bytes, c->stream>>>(a);
      return hip_ok(hipGetLastError());
    }
    return PSCLBM_EINVAL;
  }
  const bool nt = c->geom.nt_even != 0;
  if (walls) {
    if (par == 0 && nt)
      k_step<Q, PREC, 0, true, true><<<nb, BLOCK, lds_bytes, c->stream>>>(a);
    else if (par == 0)
      k_step<Q, PREC, 0, true><<<nb, BLOCK, lds_bytes, c->stream>>>(a);
    else
      k_step<Q, PREC, 1, true><<<nb, BLOCK, lds_bytes, c->stream>>>(a);
  } else {
    if (par == 0 && nt)
      k_step<Q, PREC, 0, false, true><<<nb, BLOCK, lds_bytes, c->stream>>>(a);
    else if (par == 0)
      k_step<Q, PREC, 0, false><<<nb, BLOCK, lds_bytes, c->stream>>>(a);
    else
      k_step<Q, PREC, 1, false><<<nb, BLOCK, lds_bytes, c->stream>>>(a);
  }
  return hip_ok(hipGetLastError());
}

template <int PREC>
static int dispatch_step_q(psclbm_ctx* c, const StepArgs& a, int par, size_t lds) {
  return c->geom.q == 9 ? dispatch_step<9, PREC>(c, a, par, lds)
                        : dispatch_step<19, PREC>(c, a, par, lds);
}

#define PSCLBM_DISPATCH(QV, PV, CALL)                                       \
  do {                                                                      \
    if ((QV) == 9) {                                                        \
      if ((PV) == PSCLBM_FP64) { constexpr int Q = 9, P = PSCLBM_FP64; CALL; } \
      else if ((PV) == PSCLBM_FP32) { constexpr int Q = 9, P = PSCLBM_FP32; CALL; } \
      else { constexpr int Q = 9, P = PSCLBM_FP32_FP16STORE; CALL; }        \
    } else {                                                                \
      if ((PV) == PSCLBM_FP64) { constexpr int Q = 19, P = PSCLBM_FP64; CALL; } \
      else if ((PV) == PSCLBM_FP32) { constexpr int Q = 19, P = PSCLBM_FP32; CALL; } \
      else { constexpr int Q = 19, P = PSCLBM_FP32_FP16STORE; CALL; }       \
    }                                                                       \
  } while (0)

int launch_zero(psclbm_ctx* c, void* p, size_t bytes) {
  return hip_ok(hipMemsetAsync(p, 0, bytes, c->stream));
}

int launch_init_equilibrium(psclbm_ctx* c, const double* rho, const double* u) {
  const int grid = grid_for(c->geom.N);
  PSCLBM_DISPATCH(c->geom.q, c->prec,
                  (k_set_equilibrium<Q, P><<<grid, 256, 0, c->stream>>>(c->geom, c->f, rho, u)));
  return hip_ok(hipGetLastError());
}

int launch_set_f(psclbm_ctx* c, const double* f) {
  const int grid = grid_for(c->geom.N);
  PSCLBM_DISPATCH(c->geom.q, c->prec,
                  (k_set_f<Q, P><<<grid, 256, 0, c->stream>>>(c->geom, c->f, f)));
  return hip_ok(hipGetLastError());
}

int launch_get_f(psclbm_ctx* c, double* f) {
  const int grid = grid_for(c->geom.N);
  const int par = (int)(c->steps & 1);
  PSCLBM_DISPATCH(c->geom.q, c->prec,
                  (k_get_f<Q, P><<<grid, 256, 0, c->stream>>>(c->geom, c->f, par, f, nullptr,
                                                              nullptr, 0.0, 0.0, 0.0)));
  return hip_ok(hipGetLastError());
}

int launch_get_macros(psclbm_ctx* c, double* rho, double* u) {
  const int grid = grid_for(c->geom.N);
  const int par = (int)(c->steps & 1);
  const double* F = c->cfg.body_force;
  PSCLBM_DISPATCH(c->geom.q, c->prec,
                  (k_get_f<Q, P><<<grid, 256, 0, c->stream>>>(c->geom, c->f, par, nullptr, rho, u,
                                                              F[0], F[1], F[2])));
  return hip_ok(hipGetLastError());
}

int launch_rasterize(psclbm_ctx* c, const psclbm_particles* p, bool dem_bins) {
  const int three_d = c->geom.q == 19;
  const int next = c->tile_cur ^ 1;
  DemBinOut db = dem_bin_out(c, dem_bins);
  long long blocks = ((long long)p->n + 3) / 4;
  long long clear = c->ntiles > db.nbins ? c->ntiles : db.nbins;
  const long long clear_blocks = (clear + 255) / 256;
  if (blocks < clear_blocks) blocks = clear_blocks < 4096 ? clear_blocks : 4096;
  if (blocks < 1) blocks = 1;
  k_rasterize<<<(unsigned)blocks, 256, 0, c->stream>>>(
      c->geom, p->n, three_d, c->cfg.shell_h, p->x, p->u, p->omega, p->radius, c->snap,
      c->tile_count_buf[next], c->tile_count_buf[c->tile_cur], c->tile_list,
      c->cfg.max_tile_particles, c->facc[0], c->facc[1], c->err, db);
  const int rc = hip_ok(hipGetLastError());
  if (rc) return rc;
  c->tile_cur = next;
  c->tile_count = c->tile_count_buf[next];
  if (dem_bins) dem_bins_advance(c);
  return PSCLBM_OK;
}

int launch_solid_fraction(psclbm_ctx* c, double* eps, int* ids, double* seps, int k) {
  const size_t lds = (sizeof(LdsEntry) + sizeof(double)) * (size_t)c->cfg.max_tile_particles;
  if (c->geom.q == 9)
    k_solid_fraction<2><<<c->ntiles, BLOCK, lds, c->stream>>>(
        c->geom, c->cfg.shell_h, c->np, c->cfg.max_tile_particles, c->tile_count, c->tile_list,
        c->snap, eps, ids, seps, k, c->err);
  else
    k_solid_fraction<3><<<c->ntiles, BLOCK, lds, c->stream>>>(
        c->geom, c->cfg.shell_h, c->np, c->cfg.max_tile_particles, c->tile_count, c->tile_list,
        c->snap, eps, ids, seps, k, c->err);
  return hip_ok(hipGetLastError());
}

// Arguments of one step from the context (state, forces and mass in place).
static StepArgs step_args(psclbm_ctx* c) {
  StepArgs a;
  a.g = c->geom;
  a.f = c->f;
  a.src = nullptr;
  a.tau = c->cfg.tau;
  for (int k = 0; k < 3; ++k) a.force[k] = c->cfg.body_force[k];
  a.h = c->cfg.shell_h;
  a.np = c->np;
  a.cap = c->cfg.max_tile_particles;
  a.tile_count = c->tile_count;
  a.tile_list = c->tile_list;
  a.snap = c->snap;
  const int next = c->force_buf ^ 1;
  a.facc = c->facc[next];
  a.fzero = c->facc[next ^ 1];
  a.mass_part = c->mass_part;
  a.outlet_u = c->outlet_u;
  a.face_stride = c->face_stride;
  a.err = c->err;
  a.omega = 1.0 / c->cfg.tau;
  a.inv_rho0 = 1.0 / c->geom.rho0;
  for (int k = 0; k < 3; ++k) a.force_f[k] = (float)a.force[k];
  a.omega_f = (float)a.omega;
  a.inv_rho0_f = (float)a.inv_rho0;
  a.rho0_f = (float)c->geom.rho0;
  a.tm_f = (float)(a.tau - 0.5);
  a.inlet_mask = a.outlet_mask = a.moving_mask = 0;
  for (int f = 0; f < 6; ++f) {
    if (c->geom.face[f] == PSCLBM_INLET_EQ) a.inlet_mask |= 1u << f;
    if (c->geom.face[f] == PSCLBM_OUTLET_EQ) a.outlet_mask |= 1u << f;
    if (c->geom.face[f] == PSCLBM_MOVING_WALL) a.moving_mask |= 1u << f;
  }
  a.open_mask = a.inlet_mask | a.outlet_mask;
  a.outlet_wave = outlet_wave_mask(c->geom, a.outlet_mask);
  a.original = c->cfg.weighting == PSCLBM_WEIGHT_ORIGINAL;
  a.dem_blocks = 0;
  std::memset(&a.dem, 0, sizeof(a.dem));
  a.px = a.pu = a.pr = nullptr;
  a.fc = nullptr;
  return a;
}

static size_t step_lds(const psclbm_ctx* c) {
  return c->np > 0 ? (sizeof(LdsEntry) + 6 * sizeof(double)) * (size_t)c->cfg.max_tile_particles
                   : 0;
}

int launch_step(psclbm_ctx* c) { return launch_step_contacts(c, nullptr, nullptr, nullptr, nullptr); }

int launch_step_contacts(psclbm_ctx* c, const DemArgs* dem, const double* x, const double* u,
                         const double* r) {
  const int par = (int)(c->steps & 1);
  StepArgs a = step_args(c);
  if (dem && dem->n > 0) {
    a.dem_blocks = ((dem->n + BLOCK / 64 - 1) / (BLOCK / 64) + 7) / 8 * 8;
    a.dem = *dem;
    a.px = x;
    a.pu = u;
    a.pr = r;
    a.fc = c->fcontact;
  }
  // outlets whose neighbour is in another wave: velocities before the step
  const unsigned separate = a.outlet_mask & ~a.outlet_wave;
  if (separate) {
    const double* F = c->cfg.body_force;
    dim3 grid((unsigned)grid_for(c->face_stride), 6);
    PSCLBM_DISPATCH(c->geom.q, c->prec,
                    (k_outlet_velocity<Q, P><<<grid, 256, 0, c->stream>>>(
                        c->geom, c->f, par, F[0], F[1], F[2], c->outlet_u, c->face_stride,
                        separate)));
    int rc = hip_ok(hipGetLastError());
    if (rc) return rc;
  }
  const size_t lds = step_lds(c);
  int rc;
  if (c->prec == PSCLBM_FP64)
    rc = dispatch_step_q<PSCLBM_FP64>(c, a, par, lds);
  else if (c->prec == PSCLBM_FP32)
    rc = dispatch_step_q<PSCLBM_FP32>(c, a, par, lds);
  else
    rc = dispatch_step_q<PSCLBM_FP32_FP16STORE>(c, a, par, lds);
  if (rc) return rc;
  c->force_buf ^= 1;
  c->steps += 1;
  c->mass_valid = 1;
  return PSCLBM_OK;
}

int launch_recompute(psclbm_ctx* c, const double* f0, int nsteps, double* ring) {
  StepArgs a = step_args(c);
  a.facc = nullptr;
  a.fzero = nullptr;
  a.mass_part = nullptr;
  const unsigned separate = a.outlet_mask & ~a.outlet_wave;
  const size_t lds = step_lds(c);
  const size_t QN = (size_t)c->geom.q * (size_t)c->geom.N;
  const double* F = c->cfg.body_force;
  for (int k = 0; k < nsteps; ++k) {
    const double* src = k == 0 ? f0 : ring + (size_t)(k - 1) * QN;
    if (separate) {
      dim3 grid((unsigned)grid_for(c->face_stride), 6);
      if (c->geom.q == 9)
        k_outlet_velocity<9, PSCLBM_FP64><<<grid, 256, 0, c->stream>>>(
            c->geom, src, 0, F[0], F[1], F[2], c->outlet_u, c->face_stride, separate);
      else
        k_outlet_velocity<19, PSCLBM_FP64><<<grid, 256, 0, c->stream>>>(
            c->geom, src, 0, F[0], F[1], F[2], c->outlet_u, c->face_stride, separate);
      int rc = hip_ok(hipGetLastError());
      if (rc) return rc;
    }
    a.src = src;
    a.f = ring + (size_t)k * QN;
    int rc = dispatch_step_q<PSCLBM_FP64>(c, a, 2, lds);
    if (rc) return rc;
  }
  return PSCLBM_OK;
}

int launch_mass(psclbm_ctx* c, double* h_mass) {
  // After a step the fused per-workgroup partials already hold the sum of
  // the stored state; otherwise reduce the state directly.
  if (!c->mass_valid) {
    PSCLBM_DISPATCH(c->geom.q, c->prec,
                    (k_mass_direct<Q, P><<<c->nblocks, 256, 0, c->stream>>>(c->geom, c->f,
                                                                            c->mass_part)));
    int rc0 = hip_ok(hipGetLastError());
    if (rc0) return rc0;
    c->mass_valid = 1;
  }
  double* tmp = c->scalar;
  k_reduce<<<1, 256, 0, c->stream>>>(c->mass_part, c->nblocks, tmp);
  int rc = hip_ok(hipGetLastError());
  if (rc) return rc;
  double dev = 0.0;
  rc = hip_ok(hipMemcpyAsync(&dev, tmp, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (rc) return rc;
  rc = hip_ok(hipStreamSynchronize(c->stream));
  if (rc) return rc;
  *h_mass = (double)c->geom.N * c->geom.rho0 + dev;
  return PSCLBM_OK;
}

}  // namespace psclbm
