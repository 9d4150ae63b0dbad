// DEM contact gather of the gfx950 PSC-LBM library (FP64), Sec. 2.5: the
// JKR normal force (Eqs. 25-27) with the jump-on / pull-off hysteresis (or
// Hertz's without adhesion), and optionally the sliding, twisting and
// rolling friction of Eqs. 22, 28, 29, gathered by one wave per particle
// from the DEM bins.  Used by the DEM kernel and (JKR without friction) by
// the contact workgroups of the coupled step kernel.
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
// monotonically to the root).  Returns the repulsive-positive force, and the
// contact radius a = x a0 and x in *a_out and *x_out when those are given.
__device__ inline double jkr_force(double R, double E, double gamma, double delta, double* dC,
                                   double* a_out = nullptr, double* x_out = nullptr) {
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
  if (a_out) *a_out = x * a0;
  if (x_out) *x_out = x;
  return 4.0 * FC * (x * x * x - x * s);
}

// Hertz's contact, the JKR one without adhesion: F = (4/3) E sqrt(R)
// delta^{3/2} and a = sqrt(R delta) for delta >= 0, nothing below.
__device__ inline double hertz_force(double R, double E, double delta, double* a_out) {
  const double d = delta > 0.0 ? delta : 0.0;
  *a_out = sqrt(R * d);
  return (4.0 / 3.0) * E * sqrt(R) * d * sqrt(d);
}

// Friction arguments of the standalone DEM kernel: each contact's springs
// (tangential displacement xi[3], twist angle theta, rolling displacement
// xr[3], unused) sit beside its id in the contact lists,
// [particle][max_contacts][SPRINGS].
struct FricArgs {
  const double* w;       // [n][3] spins at the start of the sub-step
  const double* prev_h;  // springs of the previous lists; null: every contact starts unloaded
  double* next_h;        // springs of the lists being built
  double k_t, eta_t, mu_f;  // sliding and twisting, with mu_f > 0
  double theta_r;           // rolling, with theta_r > 0 (and adhesion)
  double dts;               // sub-step
};

// Sliding, twisting and rolling friction on body i from one contact (Eqs.
// 22, 28, 29), each a linear spring-dashpot-slider.  n: unit normal from i
// to its partner; R: the effective radius; vr: velocity of the partner's
// surface point relative to i's at the contact; dw: i's spin minus the
// partner's; Fne: the elastic normal force (repulsive positive);
// FC = 3 pi gamma R; a: the contact radius, x = a / a0.  h holds the springs
// of the previous sub-step and receives the new ones; the force on i is
// added to f and its torque about i's centre to t.  Each stored
// displacement is first turned into the current tangent plane, then the
// sub-step's motion is added.  Sliding: a force beyond
// F_crit = mu_f |F_ne + 2 F_C| is capped, the spring reset to the stretch
// that gives the capped value; twisting likewise beyond 3 pi a F_crit / 16.
// Rolling: xr integrates v_L = R dw x n, clamped at |xr| = theta_crit R, and
// acts on i with the moment k_r (xr x n), k_r = 4 F_C x^{3/2}.
__device__ inline void contact_friction(const FricArgs& fr, double n0, double n1, double n2,
                                        double ri, double R, double vr0, double vr1, double vr2,
                                        double dw0, double dw1, double dw2, double Fne, double FC,
                                        double a, double x, double h[SPRINGS], double f[3],
                                        double t[3]) {
  if (fr.theta_r > 0.0 && FC > 0.0) {
    const double c0 = dw1 * n2 - dw2 * n1, c1 = dw2 * n0 - dw0 * n2, c2 = dw0 * n1 - dw1 * n0;
    const double hn = h[4] * n0 + h[5] * n1 + h[6] * n2;
    double r0 = h[4] - hn * n0 + fr.dts * R * c0;
    double r1 = h[5] - hn * n1 + fr.dts * R * c1;
    double r2 = h[6] - hn * n2 + fr.dts * R * c2;
    const double mag = sqrt(r0 * r0 + r1 * r1 + r2 * r2), cap = fr.theta_r * R;
    if (mag > cap) {
      const double sc = cap / mag;
      r0 *= sc;
      r1 *= sc;
      r2 *= sc;
    }
    const double kr = 4.0 * FC * x * sqrt(x);
    t[0] += kr * (r1 * n2 - r2 * n1);
    t[1] += kr * (r2 * n0 - r0 * n2);
    t[2] += kr * (r0 * n1 - r1 * n0);
    h[4] = r0;
    h[5] = r1;
    h[6] = r2;
  }
  if (!(fr.mu_f > 0.0)) return;
  const double om = -(dw0 * n0 + dw1 * n1 + dw2 * n2);
  const double vn = vr0 * n0 + vr1 * n1 + vr2 * n2;
  const double vt0 = vr0 - vn * n0, vt1 = vr1 - vn * n1, vt2 = vr2 - vn * n2;
  const double hn = h[0] * n0 + h[1] * n1 + h[2] * n2;
  double x0 = h[0] - hn * n0 + fr.dts * vt0;
  double x1 = h[1] - hn * n1 + fr.dts * vt1;
  double x2 = h[2] - hn * n2 + fr.dts * vt2;
  double F0 = fr.k_t * x0 + fr.eta_t * vt0;
  double F1 = fr.k_t * x1 + fr.eta_t * vt1;
  double F2 = fr.k_t * x2 + fr.eta_t * vt2;
  const double Fcrit = fr.mu_f * fabs(Fne + 2.0 * FC);
  const double Fm = sqrt(F0 * F0 + F1 * F1 + F2 * F2);
  if (Fm > Fcrit) {
    const double sc = Fcrit / Fm;
    F0 *= sc;
    F1 *= sc;
    F2 *= sc;
    x0 = (F0 - fr.eta_t * vt0) / fr.k_t;
    x1 = (F1 - fr.eta_t * vt1) / fr.k_t;
    x2 = (F2 - fr.eta_t * vt2) / fr.k_t;
  }
  f[0] += F0;
  f[1] += F1;
  f[2] += F2;
  t[0] += ri * (n1 * F2 - n2 * F1);  // (r_i n) x F
  t[1] += ri * (n2 * F0 - n0 * F2);
  t[2] += ri * (n0 * F1 - n1 * F0);
  const double kr = 0.5 * fr.k_t * a * a, er = 0.5 * fr.eta_t * a * a;
  double th = h[3] + fr.dts * om;
  double M = kr * th + er * om;
  const double Mcrit = 3.0 * M_PI * a * Fcrit / 16.0;
  if (fabs(M) > Mcrit) {
    M = copysign(Mcrit, M);
    th = (M - er * om) / kr;
  }
  t[0] += M * n0;
  t[1] += M * n1;
  t[2] += M * n2;
  h[0] = x0;
  h[1] = x1;
  h[2] = x2;
  h[3] = th;
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

// Contact force on particle i (position xs, velocity us, radius ri at the
// start of the sub-step), gathered by the 64 lanes of one wave: the lanes
// stride over the walls of the non-periodic axes and the (neighbour bin,
// slot) candidates, whose positions and velocities are the binning's records
// (so no particle sees another's update).  Contacts are compacted into the
// new contact list (d.next_id / d.next_n) with a ballot, and every lane
// returns the force summed over the wave in fsum.  With HERTZ the normal
// force is Hertz's (no adhesion, gamma == 0).  With FRIC, each contact also
// carries the friction of contact_friction (walls at rest; the spins are ws
// for i and fr->w for the partners, a 2D disk spinning about z only): its
// springs go beside its id into fr->next_h and the torque summed over the
// wave is returned in tsum.  Every lane of the wave must be active.
template <bool FRIC = false, bool HERTZ = false>
__device__ inline void dem_contact_wave(const DemArgs& d, int i, int lane, const double* xs,
                                        const double* us, double r_i, double* fsum,
                                        const FricArgs* fr = nullptr, const double* ws = nullptr,
                                        double* tsum = nullptr) {
  const int D = d.three_d ? 3 : 2;
  // the particle's own values are the same in every lane (scalar registers)
  const double ri = wave_uniform(r_i);
  const double xi0 = wave_uniform(xs[0]), xi1 = wave_uniform(xs[1]);
  const double xi2 = d.three_d ? wave_uniform(xs[2]) : 0.0;
  const double ui0 = wave_uniform(us[0]), ui1 = wave_uniform(us[1]);
  const double ui2 = d.three_d ? wave_uniform(us[2]) : 0.0;
  double wi0 = 0.0, wi1 = 0.0, wi2 = 0.0;
  if constexpr (FRIC) {
    wi2 = wave_uniform(ws[2]);
    if (d.three_d) {
      wi0 = wave_uniform(ws[0]);
      wi1 = wave_uniform(ws[1]);
    }
  }
  // the previous contact list, one entry per lane (max_contacts <= 64)
  const int pn = __builtin_amdgcn_readfirstlane(d.prev_n[i]);
  const int pid = lane < d.max_contacts ? d.prev_id[(size_t)i * d.max_contacts + lane] : 0;
  auto was_in_contact = [&](int id) {
    bool hit = false;
    for (int k = 0; k < pn; ++k) hit |= __builtin_amdgcn_readlane(pid, k) == id;
    return hit;
  };
  // with friction: the position of id in the previous list, or -1
  auto prev_slot = [&](int id) {
    int at = -1;
    for (int k = 0; k < pn; ++k)
      if (__builtin_amdgcn_readlane(pid, k) == id) at = k;
    return at;
  };
  // the springs of previous-list entry k (zero for a new contact)
  auto load_springs = [&](int k, double h[SPRINGS]) {
    if (k >= 0 && fr->prev_h) {
      const double* hp = fr->prev_h + ((size_t)i * d.max_contacts + k) * SPRINGS;
      for (int b = 0; b < SPRINGS; ++b) h[b] = hp[b];
    } else {
      for (int b = 0; b < SPRINGS; ++b) h[b] = 0.0;
    }
  };
  // elastic normal force and delta_C, with the contact radius and x = a / a0
  // when friction needs them
  auto normal_force = [&](double R, double delta, double* dC, double* acon, double* xcon) {
    if constexpr (HERTZ) {
      *dC = 0.0;
      *xcon = 0.0;
      return hertz_force(R, d.E, delta, acon);
    } else {
      return jkr_force(R, d.E, d.gamma, delta, dC, FRIC ? acon : nullptr,
                       FRIC ? xcon : nullptr);
    }
  };
  int* next = d.next_id + (size_t)i * d.max_contacts;
  double fs0 = 0.0, fs1 = 0.0, fs2 = 0.0;
  double tq[3] = {0.0, 0.0, 0.0};
  double h[SPRINGS] = {};
  auto store = [&](bool have, int id, unsigned long long m, int cnt) {
    if (have) {
      const int pos = cnt + lanes_below(m);
      if (pos < d.max_contacts) {
        next[pos] = id;
        if constexpr (FRIC) {
          double* hn = fr->next_h + ((size_t)i * d.max_contacts + pos) * SPRINGS;
          for (int b = 0; b < SPRINGS; ++b) hn[b] = h[b];
        }
      }
    }
  };
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
        int kp = -1;
        bool touch;
        if constexpr (FRIC) {
          kp = prev_slot(id);
          touch = delta >= 0.0 || kp >= 0;
        } else {
          touch = delta >= 0.0 || was_in_contact(id);
        }
        if (touch) {
          const double sgn = (face % 2 == 0) ? -1.0 : 1.0;  // normal towards the wall
          const double damp = d.eta_n * (-ua * sgn);
          double dC, acon, xcon;
          const double F = normal_force(ri, delta, &dC, &acon, &xcon);
          if (delta >= 0.0 || delta > -dC) {
            const double fm = (-F + damp) * sgn;
            if (a == 0) fs0 += fm;
            else if (a == 1) fs1 += fm;
            else fs2 += fm;
            have = true;
            if constexpr (FRIC) {
              const double n0 = a == 0 ? sgn : 0.0, n1 = a == 1 ? sgn : 0.0,
                           n2 = a == 2 ? sgn : 0.0;
              // the wall is at rest: vr = -(u_i + omega_i x (r_i n))
              const double vr0 = -(ui0 + ri * (wi1 * n2 - wi2 * n1));
              const double vr1 = -(ui1 + ri * (wi2 * n0 - wi0 * n2));
              const double vr2 = -(ui2 + ri * (wi0 * n1 - wi1 * n0));
              double f[3] = {0.0, 0.0, 0.0};
              load_springs(kp, h);
              contact_friction(*fr, n0, n1, n2, ri, ri, vr0, vr1, vr2, wi0, wi1, wi2, F,
                               3.0 * M_PI * d.gamma * ri, acon, xcon, h, f, tq);
              fs0 += f[0];
              fs1 += f[1];
              fs2 += f[2];
            }
          }
        }
      }
    }
    const unsigned long long m = __ballot(have);
    store(have, id, m, cnt);
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
        int kp = -1;
        bool touch;
        if constexpr (FRIC) {
          kp = prev_slot(j);
          touch = delta >= 0.0 || kp >= 0;
        } else {
          touch = delta >= 0.0 || was_in_contact(j);
        }
        if (touch) {
          // normal and normal relative velocity first: only they (and the
          // force sums) stay live across the JKR solve
          const double inv = 1.0 / dist;
          const double n0 = dv0 * inv, n1 = dv1 * inv, n2 = dv2 * inv;
          double vrn = (rc[3] - ui0) * n0 + (rc[4] - ui1) * n1;
          if (d.three_d) vrn += (rc[5] - ui2) * n2;
          const double damp = d.eta_n * vrn;
          const double Reff = 1.0 / (1.0 / ri + 1.0 / rj);
          double dC, acon, xcon;
          const double F = normal_force(Reff, delta, &dC, &acon, &xcon);
          if (delta >= 0.0 || delta > -dC) {
            const double fm = -F + damp;
            fs0 += fm * n0;
            fs1 += fm * n1;
            fs2 += fm * n2;
            have = true;
            id = j;
            if constexpr (FRIC) {
              const double uj2 = d.three_d ? rc[5] : 0.0;
              const double wj2 = fr->w[3 * j + 2];
              const double wj0 = d.three_d ? fr->w[3 * j] : 0.0;
              const double wj1 = d.three_d ? fr->w[3 * j + 1] : 0.0;
              // (u_j + omega_j x (-r_j n)) - (u_i + omega_i x (r_i n))
              const double vr0 = (rc[3] - ui0) - rj * (wj1 * n2 - wj2 * n1) -
                                 ri * (wi1 * n2 - wi2 * n1);
              const double vr1 = (rc[4] - ui1) - rj * (wj2 * n0 - wj0 * n2) -
                                 ri * (wi2 * n0 - wi0 * n2);
              const double vr2 = (uj2 - ui2) - rj * (wj0 * n1 - wj1 * n0) -
                                 ri * (wi0 * n1 - wi1 * n0);
              double f[3] = {0.0, 0.0, 0.0};
              load_springs(kp, h);
              contact_friction(*fr, n0, n1, n2, ri, Reff, vr0, vr1, vr2, wi0 - wj0, wi1 - wj1,
                               wi2 - wj2, F, 3.0 * M_PI * d.gamma * Reff, acon, xcon, h, f, tq);
              fs0 += f[0];
              fs1 += f[1];
              fs2 += f[2];
            }
          }
        }
      }
    }
    const unsigned long long m = __ballot(have);
    store(have, id, m, cnt);
    cnt += __popcll(m);
  }
  fsum[0] = wave_sum(fs0);
  fsum[1] = wave_sum(fs1);
  fsum[2] = wave_sum(fs2);
  if constexpr (FRIC) {
    tsum[0] = wave_sum(tq[0]);
    tsum[1] = wave_sum(tq[1]);
    tsum[2] = wave_sum(tq[2]);
  }
  if (lane == 0) {
    if (cnt > d.max_contacts) {
      atomicOr(d.err, ERR_CONTACTS);
      cnt = d.max_contacts;
    }
    d.next_n[i] = cnt;
  }
}

}  // namespace psclbm
