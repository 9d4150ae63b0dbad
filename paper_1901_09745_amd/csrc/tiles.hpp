// Device helpers shared by the step and adjoint kernels: nearest-image
// arithmetic, the Table 1 pair fraction, the LDS image of a tile's particle
// list and its per-cell slot search, tile geometry, and lattice links.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.hpp"

namespace psclbm {

// Minimum-image separation along one axis, as selects (no branch): the
// same sums d - L or d + L as a branch would take, d + 0 otherwise.
__device__ __forceinline__ double min_image(double d, int periodic, int L) {
  const double Ld = (double)L;
  const double hL = 0.5 * Ld;
  double t = d > hL ? -Ld : 0.0;
  t = d < -hL ? Ld : t;
  return periodic ? d + t : d;
}

// The same in FP32 for c - xh, c an integer cell coordinate and xh the FP32
// high part of a centre in [0, L): the difference and the shift by L are
// exact (both are multiples of xh's last place and no larger than L), so the
// arm c - x = min_image(c - xh) - xl rounds once.
__device__ __forceinline__ float min_image_f(float d, int periodic, int L) {
  const float Lf = (float)L;
  const float hL = 0.5f * Lf;
  float t = d > hL ? -Lf : 0.0f;
  t = d < -hL ? Lf : t;
  return periodic ? d + t : d;
}

// ---------------------------------------------------------------------------
// Solid fraction of one (cell, particle) pair, the inside/outside rule of Table 1 with
// Eq. 15/18: eps = V_a(r) + 1/2 - d inside the shell r +- h.
// ---------------------------------------------------------------------------
__device__ inline double pair_eps(double d, double r, double cs, double h) {
  double e;
  if (d >= r + h) e = 0.0;
  else if (d <= r - h) e = 1.0;
  else e = cs - d;
  if (e <= 0.0) e = 0.0;
  if (e >= 1.0) e = 1.0;
  return e;
}

// Square root of v > 0 to FP64 accuracy from the hardware FP32 root, refined
// by one Newton step in FP64 (relative error about 1e-15: the square of the
// FP32 root's), in place of the longer correctly rounded FP64 sequence.
__device__ __forceinline__ double sqrt_nr(double v) {
  const float s = __builtin_amdgcn_sqrtf((float)v);
  const double s0 = (double)s;
  const double res = fma(-s0, s0, v);
  return s > 0.0f ? s0 + res * (double)(0.5f * __builtin_amdgcn_rcpf(s)) : 0.0;
}

// LDS image of a tile's particle list.
struct LdsEntry {
  double x, y, z;
  double r, cs;
  double u[3], w[3];
  // the centre as an FP32 pair, x = xh + xl to FP64 accuracy, and U and
  // Omega rounded to FP32: the FP32 arithmetic forms take u_s = U + Omega x r
  // from these
  float xh[3], xl[3];
  float uf[3], wf[3];
  int id;
  int pad;
};

// Slots of one cell: up to KSLOTS particles with eps > 0, ascending particle
// id (lds[e[k]].id).  The fractions are evaluated in FP64 and held as E (FP64,
// or FP32 for the FP32 arithmetic forms, whose weights are formed in FP32).
template <typename E>
struct SlotsT {
  int n;
  int e[KSLOTS];  // index in the tile list
  E eps[KSLOTS];
};
using Slots = SlotsT<double>;

// Workgroup LDS of the slot search: per cell, the slots found so far.
template <typename E>
struct SlotLdsT {
  int n[BLOCK];
  unsigned short e[KSLOTS][BLOCK];  // list entries (the list holds at most 512)
  E eps[KSLOTS][BLOCK];
};
using SlotLds = SlotLdsT<double>;

// Inclusive prefix sum of an int over the 64 lanes of a wave, in DPP steps:
// shifts by 1, 2, 4 and 8 within each row of 16 lanes, then the row totals
// carried up by the row broadcasts of lanes 15 and 31.  Every lane of the
// wave must be active.
__device__ __forceinline__ int wave_scan_incl(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15 -> rows 1, 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);  // row_bcast:31 -> rows 2, 3
  return v;
}

// The cells of one wave form one x-row of the tile (TX == 64), so a list
// entry's y and z separations are the same for the whole wave.  Phase 1: each
// lane takes one list entry and, when its shell r + h reaches the row, the
// chord of the row the shell can cover (the lanes whose cell centres lie
// within sqrt((r + h)^2 - dy^2 - dz^2) of the centre's nearest image, bounded
// in FP32 and widened by 1e-3 lanes, since it only limits the cells examined;
// on periodic x narrower than 64 + 2 (r + h) + 2 the whole row).  Phase 2: the
// (entry, cell) pairs of all chords, laid out entry by entry by a prefix scan,
// are taken 64 at a time, one per lane: Table 1 for the pair in FP64, and a
// slot of its cell in LDS when the fraction is positive.  Phase 3: each cell reads its
// slots and orders them by particle id.  At most KSLOTS slots are kept per
// cell (more set ERR_SLOTS).  All 64 lanes must call this.
static_assert(SEG == 64, "one wave per 64-cell row segment");

template <int D, typename E>
__device__ inline void collect_slots(const Geom& g, int x0, int y, int z, bool active,
                                     const LdsEntry* lds, int cnt, double h, SlotsT<E>& s,
                                     unsigned* err, SlotLdsT<E>& sl) {
  const int px = g.periodic[0], py = g.periodic[1], pz = g.periodic[2];
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int tid = (int)threadIdx.x;
  const int lane = tid & 63;
  const int wbase = tid - lane;
  const bool row = y < ny && z < nz;  // uniform over the wave
  const int xlim = (nx - 1 - x0) < 63 ? (nx - 1 - x0) : 63;
  const double Lx = (double)nx;
  const double xc = (double)x0 + 31.5;
  sl.n[tid] = 0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  for (int base = 0; row && base < cnt; base += 64) {
    // phase 1: chords
    const int ec = base + lane;
    int chord = 0, lo = 0, wrap = 0, shc = 0;
    double dyz2 = 0.0;
    if (ec < cnt) {
      const LdsEntry& P = lds[ec];
      const double dy = min_image((double)y - P.y, py, ny);
      dyz2 = dy * dy;
      if constexpr (D == 3) {
        const double dz = min_image((double)z - P.z, pz, nz);
        dyz2 += dz * dz;
      }
      const double rh = P.r + h;
      if (dyz2 < rh * rh) {
        // x-image of the centre nearest the row's middle: shc 1 is -Lx, 2 is +Lx
        const double ddx = xc - P.x;
        if (px) shc = ddx > 0.5 * Lx ? 1 : (ddx < -0.5 * Lx ? 2 : 0);
        wrap = px && Lx < 66.0 + 2.0 * rh;
        int hi;
        if (wrap) {
          lo = 0;
          hi = xlim;
        } else {
          // the chord only bounds the cells examined (their membership is
          // decided in phase 2), so FP32 with a margin of 1e-3 lanes will do
          const double sh = shc == 1 ? -Lx : (shc == 2 ? Lx : 0.0);
          const float half = __builtin_amdgcn_sqrtf((float)(rh * rh - dyz2));
          const float c0 = (float)((P.x - sh) - (double)x0);  // centre's image, in lanes
          const float l = ceilf(c0 - half - 1e-3f), u = floorf(c0 + half + 1e-3f);
          lo = l < 0.0f ? 0 : (int)l;
          hi = u > (float)xlim ? xlim : (int)u;
        }
        chord = hi >= lo ? hi - lo + 1 : 0;
      }
    }
    const int incl = wave_scan_incl(chord);
    const int off = incl - chord;
    const int total = __builtin_amdgcn_readlane(incl, 63);
    const unsigned long long cmask = __ballot(chord > 0);
    // lo (6 bits), wrap, shc (2 bits) and off in one word for the broadcast
    const int pk = lo | (wrap << 6) | (shc << 7) | (off << 9);
    // phase 2: one (entry, cell) pair per lane
    for (int jb = 0; jb < total; jb += 64) {
      const int j = jb + lane;
      int b = 0;
      for (unsigned long long m = cmask; m; m &= m - 1) {
        const int c = __ffsll(m) - 1;
        if (j >= __builtin_amdgcn_readlane(off, c)) b = c;
      }
      const int pkb = __shfl(pk, b, 64);
      const double dyz2b = __shfl(dyz2, b, 64);
      const int lob = pkb & 63, wrapb = (pkb >> 6) & 1, offb = pkb >> 9;
      const double shb = ((pkb >> 7) & 3) == 1 ? -Lx : (((pkb >> 7) & 3) == 2 ? Lx : 0.0);
      const int cl = lob + (j - offb);  // cell lane of the pair
      const bool valid = j < total && (unsigned)cl < 64u;
      const int e = base + b;
      const LdsEntry& P = lds[valid ? e : 0];
      double dx = (double)(x0 + cl) - P.x;
      dx = wrapb ? min_image(dx, px, nx) : dx + shb;
      const double d2 = dx * dx + dyz2b;
      // the Table 1 rule on d = sqrt(d2)
      const double rh = P.r + h;
      const bool in_shell = valid && d2 < rh * rh;
      double eps = 0.0;
      if constexpr (std::is_same<E, float>::value) {
        // the FP32 arithmetic forms: the refined FP32 root for every pair in
        // the shell (a wave with one lane in the band takes the root for all
        // its lanes anyway), the rule's clamps giving 0 and 1.  The fraction
        // itself stays accurate to FP64: near eps = 1 the weight B amplifies
        // its error about (1 + tau - 1/2) / (tau - 1/2) times
        if (in_shell) eps = pair_eps(sqrt_nr(d2), P.r, P.cs, h);
      } else {
        // FP64: the root only where the fraction is not already fixed at 0
        // or 1 by the shell or the clamp
        const double rl = P.r - h;
        const double c1 = P.cs - 1.0;
        const bool inner = (rl >= 0.0 && d2 <= rl * rl) || (c1 >= 0.0 && d2 <= c1 * c1);
        const bool outer = P.cs <= 0.0 || d2 >= P.cs * P.cs;
        eps = inner ? 1.0 : 0.0;
        if (in_shell && !inner && !outer) eps = pair_eps(sqrt(d2), P.r, P.cs, h);
      }
      if (in_shell && eps > 0.0) {
        const int c = wbase + cl;
        const int k = atomicAdd(&sl.n[c], 1);
        if (k < KSLOTS) {
          sl.e[k][c] = (unsigned short)e;
          sl.eps[k][c] = (E)eps;
        } else if (err) {
          atomicOr(err, ERR_SLOTS);
        }
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // phase 3: this cell's slots, in ascending particle id
  int n = sl.n[tid];
  n = n < KSLOTS ? n : KSLOTS;
  if (!active) n = 0;
  s.n = n;
#pragma unroll
  for (int k = 0; k < KSLOTS; ++k) {
    const bool has = k < n;
    s.e[k] = has ? sl.e[k][tid] : 0;
    s.eps[k] = has ? sl.eps[k][tid] : (E)0;
  }
  // the ids are read and compared only where some cell of the wave holds two
  // slots or more, and the full network only where one holds three or more
  if (__any(n > 1)) {
    int id[KSLOTS];
#pragma unroll
    for (int k = 0; k < KSLOTS; ++k) id[k] = k < n ? lds[s.e[k]].id : 0x7fffffff;
    // compare-exchange network on (id, e, eps): (0,1) (2,3) (0,2) (1,3) (1,2)
    auto cx = [&](int i, int k) {
      const bool sw = id[k] < id[i];
      const int ti = id[i], te = s.e[i];
      const E tp = s.eps[i];
      id[i] = sw ? id[k] : ti;
      s.e[i] = sw ? s.e[k] : te;
      s.eps[i] = sw ? s.eps[k] : tp;
      id[k] = sw ? ti : id[k];
      s.e[k] = sw ? te : s.e[k];
      s.eps[k] = sw ? tp : s.eps[k];
    };
    static_assert(KSLOTS == 4, "sorting network for four slots");
    cx(0, 1);
    if (__any(n > 2)) {
      cx(2, 3);
      cx(0, 2);
      cx(1, 3);
      cx(1, 2);
    }
  }
}


// Loads the tile's particle list into LDS (in list order: the slot search
// orders each cell's slots by particle id) and clears its force accumulators.
// Returns the list length (uniform over the block); when it is positive the
// block has passed a barrier after the fill.  Must be called by the whole
// block.
__device__ inline int load_tile_list(const int* tile_count, const int* tile_list, int cap,
                                     const PSnap* snap, int tile, LdsEntry* lds, double* acc,
                                     int np) {
  // each thread's first list entry is read alongside the count (entries past
  // the count are stale ids or zeros inside the list buffer, never used)
  const int* lst = tile_list + (size_t)tile * cap;
  const int e0 = (int)threadIdx.x;
  const int pre = np > 0 && e0 < cap ? lst[e0] : 0;
  int cnt = np > 0 ? tile_count[tile] : 0;
  if (cnt > cap) cnt = cap;
  if (cnt == 0) return 0;
  for (int e = e0; e < cnt; e += BLOCK) {
    const int id = e == e0 ? pre : lst[e];
    const PSnap& P = snap[id];
    LdsEntry& L = lds[e];
    L.x = P.x[0];
    L.y = P.x[1];
    L.z = P.x[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      L.xh[a] = (float)P.x[a];
      L.xl[a] = (float)(P.x[a] - (double)L.xh[a]);
      L.uf[a] = (float)P.u[a];
      L.wf[a] = (float)P.w[a];
    }
    L.r = P.r;
    L.cs = P.cs;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      L.u[a] = P.u[a];
      L.w[a] = P.w[a];
    }
    L.id = id;
  }
  if (acc)
    for (int k = threadIdx.x; k < 6 * cnt; k += BLOCK) acc[k] = 0.0;
  __syncthreads();
  return cnt;
}

// The calling wave's cells in a tile: the 64-cell row segment starting at x
// = xw in row (y, z).  The results are uniform over the wave (scalar).
__device__ inline void wave_segment(const Geom& g, int tile, int& xw, int& y, int& z) {
  const int tx = tile % g.ntx;
  const int r = tile / g.ntx;
  const int ty = r % g.nty;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int segs = g.twx >> 6;  // segments per tile row
  xw = __builtin_amdgcn_readfirstlane(tx * g.twx + SEG * (w % segs));
  y = __builtin_amdgcn_readfirstlane(ty * g.twy + w / segs);
  z = __builtin_amdgcn_readfirstlane(r / g.nty);
}


// Workgroup -> tile map.  The dispatcher deals consecutive workgroups round-
// robin to the 8 XCDs; this bijection gives each XCD one contiguous run of
// tiles so that the halo lines shared by neighbouring tiles stay in one L2.
__device__ inline int xcd_tile(int b, int nb) {
  constexpr int NX = 8;
  const int per = nb / NX, rem = nb % NX;
  const int xcd = b % NX, k = b / NX;
  return xcd * per + (xcd < rem ? xcd : rem) + k;
}
// The remap pays for 64-wide tiles, whose x-neighbours share the halo lines;
// wider tiles keep those lines inside the workgroup and run as dispatched.
__device__ inline int tile_of(const Geom& g, int b, int nb) { return g.remap ? xcd_tile(b, nb) : b; }

// Lattice extents and periodicity as plain scalars (no arrays: every access
// stays a register or a kernel-argument load).
struct Dims {
  int nx, ny, nz;
  int px, py, pz;
  unsigned sy, sz;  // strides of y and z
};

__device__ __forceinline__ Dims dims_of(const Geom& g) {
  Dims d;
  d.nx = g.nx;
  d.ny = g.ny;
  d.nz = g.nz;
  d.px = g.periodic[0];
  d.py = g.periodic[1];
  d.pz = g.periodic[2];
  d.sy = (unsigned)g.nx;
  d.sz = (unsigned)g.nx * (unsigned)g.ny;
  return d;
}

// The link from cell (x, y, z) along (dx, dy, dz): sets the neighbour's cell
// offset m (periodic wrap applied) and returns the mask of non-periodic faces
// the link leaves through (bit f for face f; 0 when the neighbour exists).
// WALLS == false: every axis is periodic and no link ever leaves.
// Offset of the neighbour e_i of a cell far from every face (no wrap, no wall).
template <typename L>
__device__ __forceinline__ unsigned link_offset(const Dims& d, int i) {
  return (unsigned)(L::ex(i) + L::ey(i) * (int)d.sy + L::ez(i) * (int)d.sz);
}

template <bool WALLS>
__device__ __forceinline__ unsigned link(const Dims& d, int x, int y, int z, int dx, int dy,
                                         int dz, unsigned n, unsigned& m) {
  unsigned out = 0;
  int off = 0;
  if (dx) {
    const int v = x + dx;
    int o = dx;
    if (v < 0) {
      if (!WALLS || d.px) o += d.nx; else out |= 1u;
    } else if (v >= d.nx) {
      if (!WALLS || d.px) o -= d.nx; else out |= 2u;
    }
    off += o;
  }
  if (dy) {
    const int v = y + dy;
    int o = dy;
    if (v < 0) {
      if (!WALLS || d.py) o += d.ny; else out |= 4u;
    } else if (v >= d.ny) {
      if (!WALLS || d.py) o -= d.ny; else out |= 8u;
    }
    off += o * (int)d.sy;
  }
  if (dz) {
    const int v = z + dz;
    int o = dz;
    if (v < 0) {
      if (!WALLS || d.pz) o += d.nz; else out |= 16u;
    } else if (v >= d.nz) {
      if (!WALLS || d.pz) o -= d.nz; else out |= 32u;
    }
    off += o * (int)d.sz;
  }
  m = (unsigned)((int)n + off);
  return WALLS ? out : 0u;
}

// ---------------------------------------------------------------------------
// Particle snapshot and tile binning (the candidate box of Table 1), shared by the
// rasterisation and by the DEM kernel that rasterises the next step.
// ---------------------------------------------------------------------------
__device__ inline double va2d(double r) {  // Eq. 19
  const double s = sqrt(r * r - 0.25);
  return 0.5 * s + r * r * atan(0.5 / s);
}
__device__ inline double va3d(double r) {  // Eq. 17 (principal-value arctangents)
  const double r2 = r * r;
  const double s = sqrt(r2 - 0.5);
  return (1.0 / 12.0 - r2) * atan(0.5 * s / (0.5 - r2)) + s / 3.0 +
         (r2 - 1.0 / 12.0) * atan(0.5 / s) - (4.0 / 3.0) * r2 * r * atan(0.25 / (r * s));
}

// Snapshot of a particle; false when the radius is outside the domain of
// Eq. 17 / 19 (the snapshot then covers no cell).  c_s = V_a(r) + 1/2 is
// taken from (r_known, cs_known) when r equals r_known (a previous snapshot
// of the same particle).
__device__ inline bool make_snap(int three_d, const double* x, const double* u, const double* w,
                                 double r, PSnap& P, double r_known = -1.0,
                                 double cs_known = 0.0) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    P.x[a] = x[a];
    P.u[a] = u[a];
    P.w[a] = w[a];
  }
  if (!three_d) {
    P.x[2] = 0.0;
    P.u[2] = 0.0;
    P.w[0] = P.w[1] = 0.0;
  }
  P.r = r;
  P.pad = 0.0;
  const bool ok = P.r * P.r > (three_d ? 0.5 : 0.25) && P.r < 1e300;
  if (!ok) {
    P.cs = -1e300;
    P.r = 0.0;
  } else if (r == r_known) {
    P.cs = cs_known;
  } else {
    P.cs = (three_d ? va3d(P.r) : va2d(P.r)) + 0.5;
  }
  return ok;
}

// Tiles touched along one axis by the cell range [lo, hi]: at most two runs
// of tile indices (the second after a periodic wrap).
struct AxisRuns {
  int a0, a1, b0, b1;  // runs [a0, a1] and [b0, b1] (b0 > b1 when absent)
};

__device__ inline AxisRuns axis_runs(int lo, int hi, int L, int T, int periodic) {
  AxisRuns r;
  r.b0 = 1;
  r.b1 = 0;
  const int nt = (L + T - 1) / T;
  if (!periodic) {
    if (lo < 0) lo = 0;
    if (hi > L - 1) hi = L - 1;
    if (lo > hi) {
      r.a0 = 1;
      r.a1 = 0;
      return r;
    }
    r.a0 = lo / T;
    r.a1 = hi / T;
    return r;
  }
  if (hi - lo + 1 >= L) {
    r.a0 = 0;
    r.a1 = nt - 1;
    return r;
  }
  const int wl = ((lo % L) + L) % L;
  const int wh = ((hi % L) + L) % L;
  if (wl <= wh) {
    r.a0 = wl / T;
    r.a1 = wh / T;
  } else {
    const int t0 = wl / T, t1 = wh / T;
    if (t1 >= t0) {
      r.a0 = 0;
      r.a1 = nt - 1;
    } else {
      r.a0 = t0;
      r.a1 = nt - 1;
      r.b0 = 0;
      r.b1 = t1;
    }
  }
  return r;
}

// Enters particle s (snapshot P) in the list of every tile of its shell box
// X +- (r + h); the 64 lanes of the calling wave stride over the tiles.
__device__ inline void bin_tiles(const Geom& g, int three_d, double h, const PSnap& P, int s,
                                 int lane, int* count, int* tile_list, int cap, unsigned* err) {
  const double R = P.r + h;
  const int L[3] = {g.nx, g.ny, g.nz};
  const int T[3] = {g.twx, g.twy, 1};
  AxisRuns runs[3];
  int la[3], lt[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int lo, hi;
    if (a == 2 && !three_d) {
      lo = hi = 0;
    } else {
      lo = (int)ceil(P.x[a] - R);
      hi = (int)floor(P.x[a] + R);
    }
    runs[a] = axis_runs(lo, hi, L[a], T[a], g.periodic[a]);
    la[a] = runs[a].a1 >= runs[a].a0 ? runs[a].a1 - runs[a].a0 + 1 : 0;
    lt[a] = la[a] + (runs[a].b1 >= runs[a].b0 ? runs[a].b1 - runs[a].b0 + 1 : 0);
  }
  const int total = lt[0] * lt[1] * lt[2];
  for (int k = lane; k < total; k += 64) {
    const int ix = k % lt[0];
    const int iy = (k / lt[0]) % lt[1];
    const int iz = k / (lt[0] * lt[1]);
    const int tx = ix < la[0] ? runs[0].a0 + ix : runs[0].b0 + (ix - la[0]);
    const int ty = iy < la[1] ? runs[1].a0 + iy : runs[1].b0 + (iy - la[1]);
    const int tz = iz < la[2] ? runs[2].a0 + iz : runs[2].b0 + (iz - la[2]);
    const int t = tx + g.ntx * (ty + g.nty * tz);
    const int slot = atomicAdd(&count[t], 1);
    if (slot < cap)
      tile_list[(size_t)t * cap + slot] = s;
    else
      atomicOr(err, ERR_SLOTS);
  }
}

// DEM bin of a position along axis a (uniform bins of width bin_size).
__device__ inline int dem_bin_coord(double x, int L, int periodic, int nbin, double bin_size) {
  double v = x;
  if (periodic) {
    v = fmod(v, (double)L);
    if (v < 0) v += L;
  }
  int b = (int)floor(v / bin_size);
  if (b < 0) b = 0;
  if (b >= nbin) b = nbin - 1;
  return b;
}

// Enters particle s (position x, velocity u, radius r) in its DEM bin of the
// target set with its record; called by one lane per particle.
__device__ inline void dem_bin_insert(const DemBinOut& b, int three_d, const Geom& g, int s,
                                      const double* x, const double* u, double r,
                                      unsigned* err) {
  const int bx = dem_bin_coord(x[0], g.nx, g.periodic[0], b.nbin[0], b.bin_size[0]);
  const int by = dem_bin_coord(x[1], g.ny, g.periodic[1], b.nbin[1], b.bin_size[1]);
  const int bz = three_d ? dem_bin_coord(x[2], g.nz, g.periodic[2], b.nbin[2], b.bin_size[2]) : 0;
  const int bin = bx + b.nbin[0] * (by + b.nbin[1] * bz);
  const int k = atomicAdd(&b.count[bin], 1);
  if (k < b.bin_cap) {
    double* rc = b.rec + ((size_t)bin * b.bin_cap + k) * 8;
    rc[0] = x[0];
    rc[1] = x[1];
    rc[2] = x[2];
    rc[3] = u[0];
    rc[4] = u[1];
    rc[5] = u[2];
    rc[6] = r;
    rc[7] = (double)s;
  } else {
    atomicOr(err, ERR_CONTACTS);
  }
}

}  // namespace psclbm
