// Device helpers shared by the step and adjoint kernels: nearest-image
// arithmetic, the Table 1 pair fraction, the LDS image of a tile's particle
// list and its per-cell slot search, tile geometry, and lattice links.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace psclbm {

// Minimum-image separation along one axis.
__device__ inline double min_image(double d, int periodic, int L) {
  if (periodic) {
    if (d > 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
  }
  return d;
}

// ---------------------------------------------------------------------------
// Solid fraction of one (cell, particle) pair, Table 1 Steps 2-4 with
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

// LDS image of a tile's particle list.
struct LdsEntry {
  double x, y, z;
  double r, cs;
  double u[3], w[3];
  int id;
  int pad;
};

// Slots of one cell: up to KSLOTS particles with eps > 0, ascending id.
struct Slots {
  int n;
  int id[KSLOTS];
  int e[KSLOTS];  // index in the tile list
  double eps[KSLOTS];
};

// The cells of one wave form one x-row of the tile (TX == 64): the wave
// first keeps the list entries whose shell r + h reaches the row (a ballot
// over the list, conservative), then each cell tests only those.  All 64
// lanes must call this (active == false for cells outside the lattice).
static_assert(TX == 64, "one wave per tile row");

template <int D>
__device__ inline void collect_slots(const Geom& g, int x0, int x, int y, int z, bool active,
                                     const LdsEntry* lds, int cnt, double h, Slots& s,
                                     unsigned* err) {
  s.n = 0;
  const int px = g.periodic[0], py = g.periodic[1], pz = g.periodic[2];
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int lane = (int)(threadIdx.x & 63);
  const double xc = (double)x0 + 31.5;
  for (int base = 0; base < cnt; base += 64) {
    const int ec = base + lane;
    bool cand = false;
    if (ec < cnt) {
      const LdsEntry& P = lds[ec];
      const double rh = P.r + h;
      const double dy = min_image((double)y - P.y, py, ny);
      double r2 = dy * dy;
      if constexpr (D == 3) {
        const double dz = min_image((double)z - P.z, pz, nz);
        r2 += dz * dz;
      }
      if (r2 < rh * rh) {
        const double half = sqrt(rh * rh - r2);
        cand = fabs(min_image(xc - P.x, px, nx)) < 31.5 + half + 1e-6;
      }
    }
    unsigned long long mask = __ballot(cand);
    while (mask) {
      const int b = __ffsll(mask) - 1;
      mask &= mask - 1;
      if (!active) continue;
      const int e = base + b;
      const LdsEntry& P = lds[e];
      const double dx = min_image((double)x - P.x, px, nx);
      const double dy = min_image((double)y - P.y, py, ny);
      double d2 = dx * dx + dy * dy;
      if constexpr (D == 3) {
        const double dz = min_image((double)z - P.z, pz, nz);
        d2 += dz * dz;
      }
      const double rh = P.r + h;
      if (!(d2 < rh * rh)) continue;
      // Table 1 Steps 3-4 on d = sqrt(d2); the root is taken only when the
      // fraction is not already fixed at 0 or 1 by the shell or the clamp
      double eps;
      const double rl = P.r - h;
      const double c1 = P.cs - 1.0;
      if (rl >= 0.0 && d2 <= rl * rl) {
        eps = 1.0;
      } else if (c1 >= 0.0 && d2 <= c1 * c1) {
        eps = 1.0;
      } else if (P.cs <= 0.0 || d2 >= P.cs * P.cs) {
        eps = 0.0;
      } else {
        eps = pair_eps(sqrt(d2), P.r, P.cs, h);
      }
      if (!(eps > 0.0)) continue;
      if (s.n >= KSLOTS) {
        if (err) atomicOr(err, ERR_SLOTS);
        continue;
      }
      // the list is in ascending id, so slots are appended in id order
#pragma unroll
      for (int j = 0; j < KSLOTS; ++j)
        if (j == s.n) {
          s.id[j] = P.id;
          s.e[j] = e;
          s.eps[j] = eps;
        }
      s.n += 1;
    }
  }
}


// Loads the tile's particle list into LDS in ascending particle id (a rank
// sort; ids in a list are distinct) and clears its force accumulators.
// Returns the list length (uniform over the block).  Must be called by the
// whole block.
__device__ inline int load_tile_list(const int* tile_count, const int* tile_list, int cap,
                                     const PSnap* snap, int tile, LdsEntry* lds, double* acc,
                                     int np) {
  int cnt = np > 0 ? tile_count[tile] : 0;
  if (cnt > cap) cnt = cap;
  if (cnt == 0) return 0;
  int* ids = reinterpret_cast<int*>(acc ? acc : reinterpret_cast<double*>(lds + cap));
  for (int e = threadIdx.x; e < cnt; e += BLOCK) ids[e] = tile_list[(size_t)tile * cap + e];
  __syncthreads();
  for (int e = threadIdx.x; e < cnt; e += BLOCK) {
    const int id = ids[e];
    int rank = 0;
    for (int j = 0; j < cnt; ++j) rank += ids[j] < id;
    const PSnap& P = snap[id];
    LdsEntry& L = lds[rank];
    L.x = P.x[0];
    L.y = P.x[1];
    L.z = P.x[2];
    L.r = P.r;
    L.cs = P.cs;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      L.u[a] = P.u[a];
      L.w[a] = P.w[a];
    }
    L.id = id;
  }
  __syncthreads();
  if (acc)
    for (int k = threadIdx.x; k < 6 * cnt; k += BLOCK) acc[k] = 0.0;
  return cnt;
}

__device__ inline void tile_origin(const Geom& g, int tile, int& x0, int& y0, int& z0) {
  const int tx = tile % g.ntx;
  const int r = tile / g.ntx;
  const int ty = r % g.nty;
  const int tz = r / g.nty;
  x0 = tx * TX;
  y0 = ty * TY;
  z0 = tz * TZ;
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

}  // namespace psclbm
