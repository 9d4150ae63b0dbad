// DEM contact gather of the gfx950 PSC-LBM library (FP64), Sec. 2.5: the
// JKR normal force (Eqs. 25-27) with the jump-on / pull-off hysteresis,
// gathered by one wave per particle from the DEM bins.  Used by the DEM
// kernel and by the contact workgroups of the coupled step kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "common.hpp"
#include "tiles.hpp"

namespace psclbm {

__device__ inline double min_img(double d, int periodic, int L) {
  if (periodic) {
    if (d > 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
  }
  return d;
}

// JKR (work of adhesion 2 gamma): F/F_C = 4 (x^3 - x^{3/2}) with x = a/a0 on
// the stable branch of delta/delta_C = 6^{1/3} (2 x^2 - (4/3) x^{1/2}),
// F_C = 3 pi gamma R, a0^3 = 9 pi gamma R^2 / E, delta_C = a0^2/(2 6^{1/3} R).
// Solved for s = x^{1/2} by Newton from above (g(s) = 2 s^4 - 4/3 s is convex
// and increasing on the branch s >= 6^{-1/3}, so the iterates decrease
// monotonically to the root).  Returns the repulsive-positive force.
__device__ inline double jkr_force(double R, double E, double gamma, double delta, double* dC) {
  const double c6 = 1.8171205928321397;  // 6^{1/3}
  const double FC = 3.0 * M_PI * gamma * R;
  const double a0 = cbrt(9.0 * M_PI * gamma * R * R / E);
  const double dc = a0 * a0 / (2.0 * c6 * R);
  *dC = dc;
  const double target = (delta / dc) / c6;
  const double sC = 1.0 / c6;
  double s;
  if (target <= 2.0 * sC * sC * sC * sC - (4.0 / 3.0) * sC) {
    s = sC;
  } else {
    s = fmax(1.0, sqrt(sqrt(1.5 * fmax(target, 0.0))));
    for (int it = 0; it < 200; ++it) {
      const double s3 = s * s * s;
      const double gs = 2.0 * s3 * s - (4.0 / 3.0) * s - target;
      const double dg = 8.0 * s3 - 4.0 / 3.0;
      double sn = s - gs / dg;
      if (sn < sC) sn = sC;
      if (!(sn < s)) break;  // monotone from above: stop when it no longer decreases
      s = sn;
    }
  }
  const double x = s * s;
  return 4.0 * FC * (x * x * x - x * s);
}

__device__ inline int bin_coord(double x, int a, const DemArgs& d) {
  return dem_bin_coord(x, d.L[a], d.periodic[a], d.nbin[a], d.bin_size[a]);
}

// Neighbour bins along one axis of bin b: cnt distinct coordinates
// first, first + 1, .. (modulo nb on a periodic axis).
struct AxisNb {
  int first, cnt, nb, periodic;
  __device__ int at(int k) const { return periodic ? (first + k) % nb : first + k; }
};

__device__ inline AxisNb axis_nb(int b, int a, const DemArgs& d) {
  AxisNb r;
  r.nb = d.nbin[a];
  r.periodic = d.periodic[a];
  if (r.periodic) {
    r.cnt = r.nb < 3 ? r.nb : 3;
    r.first = r.nb < 3 ? b : b - 1 + r.nb;
  } else {
    r.first = b > 0 ? b - 1 : 0;
    r.cnt = (b + 1 < r.nb ? b + 1 : r.nb - 1) - r.first + 1;
  }
  return r;
}

// Contact force on particle i (position xs, velocity us, radius ri at the
// start of the sub-step), gathered by the 64 lanes of one wave: the lanes
// stride over the walls of the non-periodic axes and the (neighbour bin,
// slot) candidates, whose positions and velocities are the binning's records
// (so no particle sees another's update).  Contacts are compacted into the
// new contact list (d.next_id / d.next_n) with a ballot, and every lane
// returns the force summed over the wave in fsum.  Every lane of the wave
// must be active.
__device__ __forceinline__ double wave_uniform(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

__device__ inline AxisNb wave_uniform(AxisNb a) {
  a.first = __builtin_amdgcn_readfirstlane(a.first);
  a.cnt = __builtin_amdgcn_readfirstlane(a.cnt);
  a.nb = __builtin_amdgcn_readfirstlane(a.nb);
  a.periodic = __builtin_amdgcn_readfirstlane(a.periodic);
  return a;
}

__device__ inline void dem_contact_wave(const DemArgs& d, int i, int lane, const double* xs,
                                        const double* us, double r_i, double* fsum) {
  const int D = d.three_d ? 3 : 2;
  // the particle's own values are the same in every lane (scalar registers)
  const double ri = wave_uniform(r_i);
  const double xi0 = wave_uniform(xs[0]), xi1 = wave_uniform(xs[1]);
  const double xi2 = d.three_d ? wave_uniform(xs[2]) : 0.0;
  const double ui0 = wave_uniform(us[0]), ui1 = wave_uniform(us[1]);
  const double ui2 = d.three_d ? wave_uniform(us[2]) : 0.0;
  // the previous contact list, one entry per lane (max_contacts <= 64)
  const int pn = __builtin_amdgcn_readfirstlane(d.prev_n[i]);
  const int pid = lane < d.max_contacts ? d.prev_id[(size_t)i * d.max_contacts + lane] : 0;
  auto was_in_contact = [&](int id) {
    bool hit = false;
    for (int k = 0; k < pn; ++k) hit |= __builtin_amdgcn_readlane(pid, k) == id;
    return hit;
  };
  int* next = d.next_id + (size_t)i * d.max_contacts;
  double fs0 = 0.0, fs1 = 0.0, fs2 = 0.0;
  int cnt = 0;  // uniform over the wave

  // walls of non-periodic axes: flat bodies at -1/2 and L-1/2 (1/R = 1/r)
  {
    bool have = false;
    int id = 0;
    if (lane < 2 * D) {
      const int face = lane, a = face / 2;
      if (!d.periodic[a]) {
        const double xa = a == 0 ? xi0 : (a == 1 ? xi1 : xi2);
        const double ua = a == 0 ? ui0 : (a == 1 ? ui1 : ui2);
        const double dist = (face % 2 == 0) ? xa + 0.5 : (d.L[a] - 0.5) - xa;
        const double delta = ri - dist;
        id = -1 - face;
        if (delta >= 0.0 || was_in_contact(id)) {
          const double sgn = (face % 2 == 0) ? -1.0 : 1.0;  // normal towards the wall
          const double damp = d.eta_n * (-ua * sgn);
          double dC;
          const double F = jkr_force(ri, d.E, d.gamma, delta, &dC);
          if (delta >= 0.0 || delta > -dC) {
            const double fm = (-F + damp) * sgn;
            if (a == 0) fs0 += fm;
            else if (a == 1) fs1 += fm;
            else fs2 += fm;
            have = true;
          }
        }
      }
    }
    const unsigned long long m = __ballot(have);
    if (have) {
      const int pos = cnt + lanes_below(m);
      if (pos < d.max_contacts) next[pos] = id;
    }
    cnt += __popcll(m);
  }

  // particle pairs from the neighbouring bins: the lanes take the
  // (neighbour bin, slot) candidates 64 at a time
  const AxisNb ax = wave_uniform(axis_nb(bin_coord(xi0, 0, d), 0, d));
  const AxisNb ay = wave_uniform(axis_nb(bin_coord(xi1, 1, d), 1, d));
  AxisNb az;
  az.first = 0;
  az.cnt = 1;
  az.nb = 1;
  az.periodic = 0;
  if (d.three_d) az = wave_uniform(axis_nb(bin_coord(xi2, 2, d), 2, d));
  const int nb = ax.cnt * ay.cnt * az.cnt;
  for (int base = 0;; base += 64) {
    const int c = base + lane;
    const int k = c % nb, slot = c / nb;
    const int kx = k % ax.cnt, ky = (k / ax.cnt) % ay.cnt, kz = k / (ax.cnt * ay.cnt);
    const int b = ax.at(kx) + d.nbin[0] * (ay.at(ky) + d.nbin[1] * az.at(kz));
    int mcount = d.bin_count[b];
    if (mcount > d.bin_cap) mcount = d.bin_cap;
    const bool valid = slot < mcount;
    if (!__any(valid)) break;
    bool have = false;
    int id = 0;
    if (valid) {
      const double* rc = d.bin_rec + ((size_t)b * d.bin_cap + slot) * 8;
      const int j = (int)rc[7];
      if (j != i) {
        const double dv0 = min_img(rc[0] - xi0, d.periodic[0], d.L[0]);
        const double dv1 = min_img(rc[1] - xi1, d.periodic[1], d.L[1]);
        const double dv2 = d.three_d ? min_img(rc[2] - xi2, d.periodic[2], d.L[2]) : 0.0;
        const double dist = sqrt(dv0 * dv0 + dv1 * dv1 + dv2 * dv2);
        const double rj = rc[6];
        const double delta = ri + rj - dist;
        if (delta >= 0.0 || was_in_contact(j)) {
          // normal and normal relative velocity first: only they (and the
          // force sums) stay live across the JKR solve
          const double inv = 1.0 / dist;
          const double n0 = dv0 * inv, n1 = dv1 * inv, n2 = dv2 * inv;
          double vrn = (rc[3] - ui0) * n0 + (rc[4] - ui1) * n1;
          if (d.three_d) vrn += (rc[5] - ui2) * n2;
          const double damp = d.eta_n * vrn;
          const double Reff = 1.0 / (1.0 / ri + 1.0 / rj);
          double dC;
          const double F = jkr_force(Reff, d.E, d.gamma, delta, &dC);
          if (delta >= 0.0 || delta > -dC) {
            const double fm = -F + damp;
            fs0 += fm * n0;
            fs1 += fm * n1;
            fs2 += fm * n2;
            have = true;
            id = j;
          }
        }
      }
    }
    const unsigned long long m = __ballot(have);
    if (have) {
      const int pos = cnt + lanes_below(m);
      if (pos < d.max_contacts) next[pos] = id;
    }
    cnt += __popcll(m);
  }
  fsum[0] = wave_sum(fs0);
  fsum[1] = wave_sum(fs1);
  fsum[2] = wave_sum(fs2);
  if (lane == 0) {
    if (cnt > d.max_contacts) {
      atomicOr(d.err, ERR_CONTACTS);
      cnt = d.max_contacts;
    }
    d.next_n[i] = cnt;
  }
}

}  // namespace psclbm
