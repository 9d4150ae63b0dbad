// Hand-written adjoint of one PSC-LBM step (FP64), the transpose of the
// per-cell Jacobian of the step of lbm.hip applied to a given sensitivity.
//
// Notation per cell n (all FP64): f the state entering the step (after the
// inlet / outlet reset), lam*_i = dJ/df*_i the sensitivity of the post-
// collision population (read where that population streams to), B_n and the
// per-particle shares B_s (Eq. 13 with the clamped cell total of Table 1), and
//   f*_i = f_i - (1 - B_n) [w (f_i - f^eq_i) - F_i]
//          + sum_s B_s [f_{-i} - f^eq_{-i}(rho,u) + f^eq_i(rho,u_s) - f_i]   (Eqs. 10, 12)
//   m_s  = B_s [rho (u_s - u) + F],  F_s -= m_s,  T_s -= r_s x m_s       (Eq. 14)
// with w = 1/tau, rho = sum f, u = (sum f e + F/2)/rho (Eq. 5),
// u_s = U_s + Omega_s x r_s, r_s = x_n - X_s (nearest image), and the Table 1
// fraction eps_s = V_a(r) + 1/2 - |r_s| inside its linear band.
// Given dJ/dF_s and dJ/dT_s (the seeds of this step), q_s = dJ/dm_s =
// -dJ/dF_s - dJ/dT_s x r_s.  Then
//   lam_j = alpha lam*_j + B_n lam*_{-j} + kappa + a_rho + a_u . (e_j - u)/rho
// with alpha = 1 - (1 - B_n) w - B_n, kappa the moving-wall term and
//   a_rho = sum_i lam*_i [(1-B_n) w f^eq_i - B_n f^eq_{-i} + sum_s B_s f^eq_i(u_s)] / rho
//           + sum_s B_s q_s . (u_s - u)
//   a_u   = sum_i lam*_i [(1-B_n) w df^eq_i/du - B_n df^eq_{-i}/du + (1-B_n) dF_i/du]
//           - sum_s B_s rho q_s
// and for each covering particle
//   dJ/du_s = B_s [sum_i lam*_i rho w_i (3 e_i + 9 (e_i.u_s) e_i - 3 u_s) + rho q_s]
//   dJ/deps_t = B_n'(S) (lam* . P) + c(S) G_t + c'(S) sum_s eps_s G_s,
//     P_i = w (f_i - f^eq_i) - F_i,  G_s = lam* . Omega^s + q_s . [rho (u_s - u) + F],
//     c = tm/den, c' = tm/den^2 (sum eps <= 1) or c = 1/S, c' = -1/S^2,
//     B_n' = tm (1 + tm)/den^2 (sum eps < 1) else 0, tm = tau - 1/2, den = 1 - S + tm,
//   dJ/dX_s += dJ/deps_s r_s/|r_s| (linear band only) - (dJ/du_s x Omega_s + dJ/dT_s x m_s)
//   dJ/dU_s += dJ/du_s,  dJ/dOmega_s += r_s x dJ/du_s.
// Inlet cells (reset to f^eq(rho0, u_in)) pass lam through df^eq/du_in to the
// face velocity and have zero sensitivity of their own state; outlet cells
// pass it through u of their interior neighbour (a second kernel).  Moving
// walls pass lam of the reflected population to the wall velocity.
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.hpp"
#include "tiles.hpp"

namespace psclbm {

struct AdjArgs {
  Geom g;
  double tau, omega;
  double force[3];
  double h;
  int np, cap;
  const int* tile_count;
  const int* tile_list;
  const PSnap* snap;
  const double* f;        // canonical FP64 state entering the step
  const double* lam_in;   // dJ/df(t+1), canonical
  double* lam_out;        // dJ/df(t), canonical
  const double* gF;       // dJ/dF_s of this step [3n] or null
  const double* gT;       // dJ/dT_s of this step [3n] or null
  double* gX;             // += [3n]
  double* gU;             // += [3n]
  double* gW;             // += [3n]
  double* gface;          // += [6][3]
  const double* outlet_u; // [6][face cells][3], velocity of each outlet's neighbour
  double* outlet_g;       // [6][face cells][3], dJ/du of that velocity
  long long face_stride;
  unsigned inlet_mask, outlet_mask, moving_mask;
  unsigned outlet_wave;   // outlet faces (x only) whose neighbour is in the same wave
};

template <int Q>
__device__ __forceinline__ double feq_i(int i, double rho, double ux, double uy, double uz,
                                        double uu) {
  using L = Lattice<Q>;
  const double eu = L::ex(i) * ux + L::ey(i) * uy + L::ez(i) * uz;
  return rho * L::w(i) * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

template <int Q, bool WALLS>
__global__ void __launch_bounds__(BLOCK) k_adjoint(const AdjArgs a) {
  using L = Lattice<Q>;
  constexpr int D = L::D;
  extern __shared__ double smem_d[];
  __shared__ SlotLds slot_lds;
  const Geom& G = a.g;
  const int tile = blockIdx.x;
  LdsEntry* lds = reinterpret_cast<LdsEntry*>(smem_d);
  double* acc = reinterpret_cast<double*>(lds + a.cap);  // [cap][9]
  const int cnt = load_tile_list(a.tile_count, a.tile_list, a.cap, a.snap, tile, lds, nullptr,
                                 a.np);
  if (cnt > 0) {
    for (int k = threadIdx.x; k < 9 * cnt; k += BLOCK) acc[k] = 0.0;
    __syncthreads();
  }
  // the wave's 64-cell row segment; y and z are uniform over the wave (scalar)
  int x0, y, z;
  wave_segment(G, tile, x0, y, z);
  const int x = x0 + (int)(threadIdx.x & 63);
  const bool active = x < G.nx && y < G.ny && z < G.nz;
  const unsigned N = (unsigned)G.N;
  const unsigned n = (unsigned)x + (unsigned)G.nx * ((unsigned)y + (unsigned)G.ny * (unsigned)z);
  Slots s;
  s.n = 0;
  if (cnt > 0) collect_slots<D>(G, x0, y, z, active, lds, cnt, a.h, s, nullptr, slot_lds);

  if (active) {
    Dims d;
    d.nx = G.nx; d.ny = G.ny; d.nz = G.nz;
    d.px = G.periodic[0]; d.py = G.periodic[1]; d.pz = G.periodic[2];
    d.sy = (unsigned)G.nx;
    d.sz = (unsigned)G.nx * (unsigned)G.ny;
    const double rho0 = G.rho0;
    const double F0 = a.force[0], F1 = a.force[1], F2 = a.force[2];
    const int lane = (int)(threadIdx.x & 63);

    // sensitivity of each post-collision population: where it streams to;
    // kappa is the moving-wall term -6 w_i rho (e_i . u_w): d/df_j = -6 w_i (e_i . u_w)
    double ls[Q];
    double kappa = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      unsigned m = n;
      const unsigned out = i == 0 ? 0u : link<WALLS>(d, x, y, z, L::ex(i), L::ey(i), L::ez(i), n, m);
      if (!out) {
        ls[i] = a.lam_in[(size_t)i * N + m];
      } else {
        ls[i] = a.lam_in[(size_t)L::opp(i) * N + n];
        const unsigned mw = out & a.moving_mask;
        if (mw) {
          double uw0 = 0.0, uw1 = 0.0, uw2 = 0.0;
#pragma unroll
          for (int fc = 0; fc < 6; ++fc)
            if ((mw >> fc) & 1u) {
              uw0 += G.face_u[fc][0];
              uw1 += G.face_u[fc][1];
              uw2 += G.face_u[fc][2];
            }
          kappa -= 6.0 * L::w(i) * edot(L::ex(i), L::ey(i), L::ez(i), uw0, uw1, uw2) * ls[i];
        }
      }
    }

    // the state entering the step, consumed as it loads: its moments and
    // the two sums through which it enters the adjoint, Sf = sum_i lam*_i f_i
    // and So = sum_i lam*_{-i} f_i (= sum_i lam*_i f_{-i}); an x-face outlet
    // whose interior neighbour is in this wave takes that neighbour's
    // velocity from its lane
    double rho_in = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0, Sf = 0.0, So = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double fi = a.f[(size_t)i * N + n];
      rho_in += fi;
      eacc(L::ex(i), j0, fi);
      eacc(L::ey(i), j1, fi);
      eacc(L::ez(i), j2, fi);
      Sf += ls[i] * fi;
      So += ls[L::opp(i)] * fi;
    }
    double uin0 = 0.0, uin1 = 0.0, uin2 = 0.0;
    double wu0 = 0.0, wu1 = 0.0, wu2 = 0.0;
    if (a.outlet_wave) {
      uin0 = (j0 + 0.5 * F0) / rho_in;
      uin1 = (j1 + 0.5 * F1) / rho_in;
      uin2 = (j2 + 0.5 * F2) / rho_in;
      int src = lane;
      if ((a.outlet_wave & 1u) && x == 0) src = lane + 1;
      if ((a.outlet_wave & 2u) && x == d.nx - 1) src = lane - 1;
      wu0 = __shfl(uin0, src);
      wu1 = __shfl(uin1, src);
      wu2 = __shfl(uin2, src);
    }

    // inlet / outlet reset (as in the forward: outlets first, an inlet wins)
    int reset = 0, rface = 0;
    double ub0 = 0.0, ub1 = 0.0, ub2 = 0.0;
    double rho = rho_in, jx = j0, jy = j1, jz = j2;
    if (a.inlet_mask | a.outlet_mask) {
#pragma unroll
      for (int fc = 0; fc < 6; ++fc) {
        const bool on = fc == 0 ? x == 0 : fc == 1 ? x == d.nx - 1 : fc == 2 ? y == 0
                      : fc == 3 ? y == d.ny - 1 : fc == 4 ? z == 0 : z == d.nz - 1;
        if (((a.outlet_mask >> fc) & 1u) && on) {
          if ((a.outlet_wave >> fc) & 1u) {
            ub0 = wu0; ub1 = wu1; ub2 = wu2;
          } else {
            const unsigned k = fc < 2 ? (unsigned)y + (unsigned)d.ny * z
                                      : (fc < 4 ? (unsigned)x + (unsigned)d.nx * z
                                                : (unsigned)x + (unsigned)d.nx * y);
            const double* o = a.outlet_u + ((size_t)fc * a.face_stride + k) * 3;
            ub0 = o[0]; ub1 = o[1]; ub2 = o[2];
          }
          reset = 2;
          rface = fc;
        }
      }
#pragma unroll
      for (int fc = 0; fc < 6; ++fc) {
        const bool on = fc == 0 ? x == 0 : fc == 1 ? x == d.nx - 1 : fc == 2 ? y == 0
                      : fc == 3 ? y == d.ny - 1 : fc == 4 ? z == 0 : z == d.nz - 1;
        if (((a.inlet_mask >> fc) & 1u) && on) {
          ub0 = G.face_u[fc][0]; ub1 = G.face_u[fc][1]; ub2 = G.face_u[fc][2];
          reset = 1;
          rface = fc;
        }
      }
      if (reset) {  // the state is f^eq(rho0, u_b)
        const double uq = ub0 * ub0 + ub1 * ub1 + ub2 * ub2;
        rho = jx = jy = jz = Sf = So = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const double fi = feq_i<Q>(i, rho0, ub0, ub1, ub2, uq);
          rho += fi;
          eacc(L::ex(i), jx, fi);
          eacc(L::ey(i), jy, fi);
          eacc(L::ez(i), jz, fi);
          Sf += ls[i] * fi;
          So += ls[L::opp(i)] * fi;
        }
      }
    }

    // moving walls: d/du_w of -6 w_i rho (e_i . u_w)
    if (a.gface && a.moving_mask) {
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        unsigned m = n;
        const unsigned mw =
            link<WALLS>(d, x, y, z, L::ex(i), L::ey(i), L::ez(i), n, m) & a.moving_mask;
        if (!mw) continue;
        const double cw = -6.0 * L::w(i) * rho * ls[i];
#pragma unroll
        for (int fc = 0; fc < 6; ++fc)
          if ((mw >> fc) & 1u) {
            if (L::ex(i)) atomicAdd(a.gface + 3 * fc, cw * L::ex(i));
            if (L::ey(i)) atomicAdd(a.gface + 3 * fc + 1, cw * L::ey(i));
            if (L::ez(i)) atomicAdd(a.gface + 3 * fc + 2, cw * L::ez(i));
          }
      }
    }

    const double ux = (jx + 0.5 * F0) / rho, uy = (jy + 0.5 * F1) / rho, uz = (jz + 0.5 * F2) / rho;
    const double uu = ux * ux + uy * uy + uz * uz;
    const double w = a.omega;
    const double kg = 1.0 - 0.5 * w;

    // weights
    double S = 0.0;
#pragma unroll
    for (int k = 0; k < KSLOTS; ++k)
      if (k < s.n) S += s.eps[k];
    const double tm = a.tau - 0.5;
    const double en = S < 1.0 ? S : 1.0;
    const double den = (1.0 - en) + tm;
    const double Bn = s.n > 0 ? en * tm / den : 0.0;
    const double c = S <= 1.0 ? tm / den : 1.0 / S;
    const double cp = S <= 1.0 ? tm / (den * den) : -1.0 / (S * S);
    const double Bnp = S < 1.0 ? tm * (1.0 + tm) / (den * den) : 0.0;

    // base adjoint terms; LP = sum_i lam*_i (w (f_i - f^eq_i) - F_i) and
    // L0 = sum_i lam*_i (f_{-i} - f^eq_{-i} - f_i), the part of lam* . Omega^s
    // common to every particle, start from the state sums Sf, So; and the
    // moments of w_i lam*_i (orders 0, 1, 2 in e_i), through which the
    // particle terms close
    // Moments of w_i lam*_i (orders 0, 1, 2 in e_i; only the nonzero
    // components of e_i are added).  Every sum over directions of the base
    // adjoint closes on them, since f^eq_i and F_i are polynomials of degree
    // two in e_i with the weight w_i, and e_{-i} = -e_i, w_{-i} = w_i:
    //   sum_i lam*_i    f^eq_i / rho = m0 (1 - 1.5 u^2) + 3 u.m1 + 4.5 u.M2.u  (Qp)
    //   sum_i lam*_{-i} f^eq_i / rho = m0 (1 - 1.5 u^2) - 3 u.m1 + 4.5 u.M2.u  (Qm)
    //   sum_i lam*_i F_i / k = 3 (F.m1 - (u.F) m0) + 9 u.M2.F
    double m0 = 0.0, m1x = 0.0, m1y = 0.0, m1z = 0.0;
    double mxx = 0.0, myy = 0.0, mzz = 0.0, mxy = 0.0, mxz = 0.0, myz = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int ex = L::ex(i), ey = L::ey(i), ez = L::ez(i);
      const double wl = L::w(i) * ls[i];
      m0 += wl;
      eacc(ex, m1x, wl);
      eacc(ey, m1y, wl);
      eacc(ez, m1z, wl);
      if (ex != 0) mxx += wl;
      if (ey != 0) myy += wl;
      if (ez != 0) mzz += wl;
      eacc(ex * ey, mxy, wl);
      eacc(ex * ez, mxz, wl);
      eacc(ey * ez, myz, wl);
    }
    const double irho = 1.0 / rho;
    const double uF = ux * F0 + uy * F1 + uz * F2;
    const double Mux = mxx * ux + mxy * uy + mxz * uz;  // M2 u
    const double Muy = mxy * ux + myy * uy + myz * uz;
    const double Muz = mxz * ux + myz * uy + mzz * uz;
    const double MFx = mxx * F0 + mxy * F1 + mxz * F2;  // M2 F
    const double MFy = mxy * F0 + myy * F1 + myz * F2;
    const double MFz = mxz * F0 + myz * F1 + mzz * F2;
    const double um1 = ux * m1x + uy * m1y + uz * m1z;
    const double uMu = ux * Mux + uy * Muy + uz * Muz;
    const double even = m0 * (1.0 - 1.5 * uu) + 4.5 * uMu;
    const double Qp = even + 3.0 * um1, Qm = even - 3.0 * um1;
    const double lF = kg * (3.0 * ((F0 * m1x + F1 * m1y + F2 * m1z) - uF * m0) +
                            9.0 * (ux * MFx + uy * MFy + uz * MFz));
    // LP = sum_i lam*_i (w (f_i - f^eq_i) - F_i) and L0 = sum_i lam*_i
    // (f_{-i} - f^eq_{-i} - f_i), the part of lam* . Omega^s common to every
    // particle, from the state sums Sf, So
    const double LP = w * (Sf - rho * Qp) - lF;
    const double L0 = So - Sf - rho * Qm;
    // the coefficient of f^eq_i is cf_i = (1-B_n) w lam*_i - B_n lam*_{-i}:
    // sum_i cf_i f^eq_i / rho, and the velocity gradient
    //   sum_i cf_i df^eq_i/du + (1-B_n) lam*_i dF_i/du
    //   = rho (3 c1 m1 + 9 c2 M2 u - 3 c2 m0 u) + (1-B_n) k (9 M2 F - 3 m0 F)
    // with c1 = (1-B_n) w + B_n, c2 = (1-B_n) w - B_n
    double ar = (1.0 - Bn) * w * Qp - Bn * Qm;
    const double c1 = (1.0 - Bn) * w + Bn, c2 = (1.0 - Bn) * w - Bn;
    const double kF = (1.0 - Bn) * kg;
    double aux = rho * (3.0 * c1 * m1x + 9.0 * c2 * Mux - 3.0 * c2 * m0 * ux) + kF * (9.0 * MFx - 3.0 * m0 * F0);
    double auy = rho * (3.0 * c1 * m1y + 9.0 * c2 * Muy - 3.0 * c2 * m0 * uy) + kF * (9.0 * MFy - 3.0 * m0 * F1);
    double auz = rho * (3.0 * c1 * m1z + 9.0 * c2 * Muz - 3.0 * c2 * m0 * uz) + kF * (9.0 * MFz - 3.0 * m0 * F2);

    // covering particles, first pass: G_s = lam* . Omega^s + q_s . M_s with
    //   lam* . f^eq(rho, u_s) = rho [m0 (1 - 1.5 u_s^2) + 3 u_s . m1 + 4.5 u_s.M2.u_s]
    //   sum_i lam*_i df^eq_i(u_s)/du_s = rho [3 m1 + 9 M2 u_s - 3 m0 u_s]
    // and every particle gradient term but the one carrying sum_s eps_s G_s;
    // dJ/deps_s = B_n' (lam* . P) + c G_s + c' sum_t eps_t G_t enters dJ/dX_s
    // through d eps / d X = r / |r| on the linear band of Table 1 (zero where
    // clamped)
    double SG = 0.0;
    const double BLP = Bnp * LP;
#pragma unroll
    for (int k = 0; k < KSLOTS; ++k) {
      if (k >= s.n) continue;
      const int e = s.e[k];
      const double epsk = s.eps[k];
      const LdsEntry& P = lds[e];
      const double rx = min_image((double)x - P.x, d.px, d.nx);
      const double ry = min_image((double)y - P.y, d.py, d.ny);
      const double rz = D == 3 ? min_image((double)z - P.z, d.pz, d.nz) : 0.0;
      const double usx = P.u[0] + P.w[1] * rz - P.w[2] * ry;
      const double usy = P.u[1] + P.w[2] * rx - P.w[0] * rz;
      const double usz = P.u[2] + P.w[0] * ry - P.w[1] * rx;
      const double us2 = usx * usx + usy * usy + usz * usz;
      const double Bs = epsk * c;
      // q = dJ/dm = -dJ/dF - dJ/dT x r
      double qx = 0.0, qy = 0.0, qz = 0.0;
      const int id = P.id;
      if (a.gF) {
        qx -= a.gF[3 * id];
        qy -= a.gF[3 * id + 1];
        qz -= a.gF[3 * id + 2];
      }
      double tx = 0.0, ty = 0.0, tz = 0.0;
      if (a.gT) {
        tx = a.gT[3 * id];
        ty = a.gT[3 * id + 1];
        tz = a.gT[3 * id + 2];
        qx -= ty * rz - tz * ry;
        qy -= tz * rx - tx * rz;
        qz -= tx * ry - ty * rx;
      }
      const double Mx = rho * (usx - ux) + F0, My = rho * (usy - uy) + F1, Mz = rho * (usz - uz) + F2;
      const double M2x = mxx * usx + mxy * usy + mxz * usz;
      const double M2y = mxy * usx + myy * usy + myz * usz;
      const double M2z = mxz * usx + myz * usy + mzz * usz;
      const double Lfs = rho * (m0 * (1.0 - 1.5 * us2) + 3.0 * (usx * m1x + usy * m1y + usz * m1z) +
                                4.5 * (usx * M2x + usy * M2y + usz * M2z));
      const double dsx = rho * (3.0 * m1x + 9.0 * M2x - 3.0 * usx * m0);
      const double dsy = rho * (3.0 * m1y + 9.0 * M2y - 3.0 * usy * m0);
      const double dsz = rho * (3.0 * m1z + 9.0 * M2z - 3.0 * usz * m0);
      const double Gs = L0 + Lfs + qx * Mx + qy * My + qz * Mz;
      SG += epsk * Gs;
      ar += Bs * Lfs / rho + Bs * (qx * (usx - ux) + qy * (usy - uy) + qz * (usz - uz));
      aux -= Bs * rho * qx;
      auy -= Bs * rho * qy;
      auz -= Bs * rho * qz;
      // dJ/du_s, and through u_s = U + Omega x r and m = B_s M: the parts of
      // dJ/dr that are dJ/du_s x Omega and dJ/dT x m
      const double ax = Bs * (dsx + rho * qx), ay = Bs * (dsy + rho * qy), az = Bs * (dsz + rho * qz);
      const double mx = Bs * Mx, my = Bs * My, mz = Bs * Mz;
      const double dist = sqrt(rx * rx + ry * ry + rz * rz);
      const double lin = P.cs - dist;
      const bool band = dist < P.r + a.h && dist > P.r - a.h && lin > 0.0 && lin < 1.0;
      const double gd = band ? (BLP + c * Gs) / dist : 0.0;
      double* ac = acc + 9 * e;
      atomicAdd(ac + 0, gd * rx - ((ay * P.w[2] - az * P.w[1]) + (ty * mz - tz * my)));
      atomicAdd(ac + 1, gd * ry - ((az * P.w[0] - ax * P.w[2]) + (tz * mx - tx * mz)));
      atomicAdd(ac + 3, ax);
      atomicAdd(ac + 4, ay);
      if constexpr (D == 3) {
        atomicAdd(ac + 2, gd * rz - ((ax * P.w[1] - ay * P.w[0]) + (tx * my - ty * mx)));
        atomicAdd(ac + 5, az);
        atomicAdd(ac + 6, ry * az - rz * ay);
        atomicAdd(ac + 7, rz * ax - rx * az);
      }
      atomicAdd(ac + 8, rx * ay - ry * ax);
    }

    // second pass: the c' sum_t eps_t G_t part of dJ/deps_s
    if (s.n > 0) {
      const double cSG = cp * SG;
#pragma unroll
      for (int k = 0; k < KSLOTS; ++k) {
        if (k >= s.n) continue;
        const int e = s.e[k];
        const LdsEntry& P = lds[e];
        const double rx = min_image((double)x - P.x, d.px, d.nx);
        const double ry = min_image((double)y - P.y, d.py, d.ny);
        const double rz = D == 3 ? min_image((double)z - P.z, d.pz, d.nz) : 0.0;
        const double dist = sqrt(rx * rx + ry * ry + rz * rz);
        const double lin = P.cs - dist;
        const bool band = dist < P.r + a.h && dist > P.r - a.h && lin > 0.0 && lin < 1.0;
        if (!band) continue;
        const double gd = cSG / dist;
        double* ac = acc + 9 * e;
        atomicAdd(ac + 0, gd * rx);
        atomicAdd(ac + 1, gd * ry);
        if constexpr (D == 3) atomicAdd(ac + 2, gd * rz);
      }
    }

    // sensitivity of the state entering the step; a reset cell passes it to
    // the boundary velocity (f = f^eq(rho0, u_b)):
    //   dJ/du_b = sum_j lam_j rho0 w_j (3 e_j + 9 (e_j.u_b) e_j - 3 u_b)
    // and keeps none of its own
    const double alpha = 1.0 - (1.0 - Bn) * w - Bn;
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    if (reset) {
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const double ex = L::ex(j), ey = L::ey(j), ez = L::ez(j);
        const double lj = alpha * ls[j] + Bn * ls[L::opp(j)] + kappa + ar +
                          (aux * (ex - ux) + auy * (ey - uy) + auz * (ez - uz)) * irho;
        const double eu = ex * ub0 + ey * ub1 + ez * ub2;
        const double rw = lj * rho0 * L::w(j);
        g0 += rw * (3.0 * ex + 9.0 * eu * ex - 3.0 * ub0);
        g1 += rw * (3.0 * ey + 9.0 * eu * ey - 3.0 * ub1);
        g2 += rw * (3.0 * ez + 9.0 * eu * ez - 3.0 * ub2);
      }
      if (reset == 1) {
        if (a.gface) {
          atomicAdd(a.gface + 3 * rface, g0);
          atomicAdd(a.gface + 3 * rface + 1, g1);
          atomicAdd(a.gface + 3 * rface + 2, g2);
        }
      } else if (!((a.outlet_wave >> rface) & 1u)) {
        const unsigned k = rface < 2 ? (unsigned)y + (unsigned)d.ny * z
                                     : (rface < 4 ? (unsigned)x + (unsigned)d.nx * z
                                                  : (unsigned)x + (unsigned)d.nx * y);
        double* o = a.outlet_g + ((size_t)rface * a.face_stride + k) * 3;
        o[0] = g0;
        o[1] = g1;
        o[2] = g2;
      }
    }
    // in-wave outlets: the neighbour lane takes the outlet's dJ/du_b through
    // its own u = (sum f e + F/2)/rho: lam_j += g . (e_j - u)/rho
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (a.outlet_wave) {
#pragma unroll
      for (int fc = 0; fc < 2; ++fc) {
        if (!((a.outlet_wave >> fc) & 1u)) continue;
        const bool mine = reset == 2 && rface == fc;
        const int nbx = fc == 0 ? 1 : d.nx - 2;
        const int src = x == nbx ? (fc == 0 ? lane - 1 : lane + 1) : lane;
        const double v0 = __shfl(mine ? g0 : 0.0, src);
        const double v1 = __shfl(mine ? g1 : 0.0, src);
        const double v2 = __shfl(mine ? g2 : 0.0, src);
        if (x == nbx) {
          s0 += v0 / rho_in;
          s1 += v1 / rho_in;
          s2 += v2 / rho_in;
        }
      }
    }
    const double sb = -(s0 * uin0 + s1 * uin1 + s2 * uin2);
    // lam_j = alpha lam*_j + B_n lam*_{-j} + kappa + ar + au.(e_j - u)/rho:
    // the part common to every j, and au/rho dotted with e_j's nonzero
    // components
    const double qx = aux * irho, qy = auy * irho, qz = auz * irho;
    const double base = kappa + ar - (qx * ux + qy * uy + qz * uz);
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int ex = L::ex(j), ey = L::ey(j), ez = L::ez(j);
      double lj = alpha * ls[j] + Bn * ls[L::opp(j)] + base + edot(ex, ey, ez, qx, qy, qz);
      if (reset) lj = 0.0;
      lj += edot(ex, ey, ez, s0, s1, s2) + sb;
      a.lam_out[(size_t)j * N + n] = lj;
    }
  }

  // flush the tile's particle gradients, one (entry, component) pair per
  // thread so that a tile's atomics are issued together
  __syncthreads();
  for (int t = threadIdx.x; t < 9 * cnt; t += BLOCK) {
    const int e = t / 9, k = t - 9 * e;
    const double v = acc[t];
    if (v == 0.0) continue;
    const int id = lds[e].id;
    double* dst = k < 3 ? a.gX : (k < 6 ? a.gU : a.gW);
    if (dst) atomicAdd(dst + 3 * id + (k % 3), v);
  }
}

// Velocity (Eq. 5) of each outlet cell's interior neighbour, from a canonical
// FP64 state.
__global__ void k_outlet_velocity_canon(Geom g, int face, const double* f, double fx, double fy,
                                        double fz, double* out, long long stride) {
  const int ax = face / 2;
  const int u1 = ax == 0 ? 1 : 0, u2 = ax == 2 ? 1 : 2;
  const int Ld[3] = {g.nx, g.ny, g.nz};
  const long long cells = (long long)Ld[u1] * Ld[u2];
  const int q = g.q;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < cells;
       k += (long long)gridDim.x * blockDim.x) {
    int p[3];
    p[u1] = (int)(k % Ld[u1]);
    p[u2] = (int)(k / Ld[u1]);
    p[ax] = (face % 2 == 0) ? 1 : Ld[ax] - 2;
    const long long m = p[0] + (long long)g.nx * (p[1] + (long long)g.ny * p[2]);
    double rho = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
    for (int i = 0; i < q; ++i) {
      const double fi = f[(size_t)i * g.N + m];
      const int ex = q == 9 ? Lattice<9>::ex(i) : Lattice<19>::ex(i);
      const int ey = q == 9 ? Lattice<9>::ey(i) : Lattice<19>::ey(i);
      const int ez = q == 9 ? Lattice<9>::ez(i) : Lattice<19>::ez(i);
      rho += fi;
      j0 += ex * fi;
      j1 += ey * fi;
      j2 += ez * fi;
    }
    double* o = out + ((size_t)face * stride + k) * 3;
    o[0] = (j0 + 0.5 * fx) / rho;
    o[1] = (j1 + 0.5 * fy) / rho;
    o[2] = (j2 + 0.5 * fz) / rho;
  }
}

// Outlet cells: the sensitivity of the reset velocity goes to the interior
// neighbour's state through u = (sum f e + F/2)/rho: lam_j += g . (e_j - u)/rho.
template <int Q>
__global__ void k_outlet_adjoint(Geom g, int face, const double* f, const double* gu,
                                 double* lam, double fx, double fy, double fz, long long stride) {
  using L = Lattice<Q>;
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
    const long long m = p[0] + (long long)g.nx * (p[1] + (long long)g.ny * p[2]);
    double rho = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
    for (int i = 0; i < Q; ++i) {
      const double fi = f[(size_t)i * g.N + m];
      rho += fi;
      j0 += L::ex(i) * fi;
      j1 += L::ey(i) * fi;
      j2 += L::ez(i) * fi;
    }
    const double ux = (j0 + 0.5 * fx) / rho, uy = (j1 + 0.5 * fy) / rho, uz = (j2 + 0.5 * fz) / rho;
    const double* gv = gu + ((size_t)face * stride + k) * 3;
    for (int j = 0; j < Q; ++j)
      lam[(size_t)j * g.N + m] +=
          (gv[0] * (L::ex(j) - ux) + gv[1] * (L::ey(j) - uy) + gv[2] * (L::ez(j) - uz)) / rho;
  }
}

// Table 1 chain alone: dJ/dX_s += sum_n dJ/deps_{n,s} r/|r| on the linear band,
// for sensitivities given per recorded slot (the order of psc_get_solid_fraction).
template <int D>
__global__ void __launch_bounds__(BLOCK) k_rasterize_adjoint(Geom g, double h, int np, int cap,
                                                           const int* tile_count,
                                                           const int* tile_list,
                                                           const PSnap* snap, const double* gs,
                                                           int kout, double* gX) {
  extern __shared__ double smem_d[];
  __shared__ SlotLds slot_lds;
  LdsEntry* lds = reinterpret_cast<LdsEntry*>(smem_d);
  const int tile = blockIdx.x;
  const int cnt = load_tile_list(tile_count, tile_list, cap, snap, tile, lds, nullptr, np);
  // the wave's 64-cell row segment; y and z are uniform over the wave (scalar)
  int x0, y, z;
  wave_segment(g, tile, x0, y, z);
  const int x = x0 + (int)(threadIdx.x & 63);
  const bool active = x < g.nx && y < g.ny && z < g.nz;
  Slots s;
  s.n = 0;
  if (cnt > 0) collect_slots<D>(g, x0, y, z, active, lds, cnt, h, s, nullptr, slot_lds);
  if (!active) return;
  const long long n = x + (long long)g.nx * (y + (long long)g.ny * z);
#pragma unroll
  for (int k = 0; k < KSLOTS; ++k) {
    if (k >= kout || k >= s.n) break;
    const double gk = gs[(size_t)n * kout + k];
    if (gk == 0.0) continue;
    const LdsEntry& P = lds[s.e[k]];
    const double rx = min_image((double)x - P.x, g.periodic[0], g.nx);
    const double ry = min_image((double)y - P.y, g.periodic[1], g.ny);
    const double rz = D == 3 ? min_image((double)z - P.z, g.periodic[2], g.nz) : 0.0;
    const double dist = sqrt(rx * rx + ry * ry + rz * rz);
    const double lin = P.cs - dist;
    if (!(dist < P.r + h && dist > P.r - h && lin > 0.0 && lin < 1.0)) continue;
    const double gd = gk / dist;
    atomicAdd(gX + 3 * P.id, gd * rx);
    atomicAdd(gX + 3 * P.id + 1, gd * ry);
    if (D == 3) atomicAdd(gX + 3 * P.id + 2, gd * rz);
  }
}

int launch_adjoint(psclbm_ctx* c, const double* f, const double* lam_in, double* lam_out,
                   const double* gF, const double* gT, double* gX, double* gU, double* gW,
                   double* gface) {
  AdjArgs a;
  a.g = c->geom;
  a.tau = c->cfg.tau;
  a.omega = 1.0 / c->cfg.tau;
  for (int k = 0; k < 3; ++k) a.force[k] = c->cfg.body_force[k];
  a.h = c->cfg.shell_h;
  a.np = c->np;
  a.cap = c->cfg.max_tile_particles;
  a.tile_count = c->tile_count;
  a.tile_list = c->tile_list;
  a.snap = c->snap;
  a.f = f;
  a.lam_in = lam_in;
  a.lam_out = lam_out;
  a.gF = gF;
  a.gT = gT;
  a.gX = gX;
  a.gU = gU;
  a.gW = gW;
  a.gface = gface;
  a.outlet_u = c->outlet_u;
  a.outlet_g = c->outlet_g;
  a.face_stride = c->face_stride;
  a.inlet_mask = a.outlet_mask = a.moving_mask = 0;
  for (int fc = 0; fc < 6; ++fc) {
    if (c->geom.face[fc] == PSCLBM_INLET_EQ) a.inlet_mask |= 1u << fc;
    if (c->geom.face[fc] == PSCLBM_OUTLET_EQ) a.outlet_mask |= 1u << fc;
    if (c->geom.face[fc] == PSCLBM_MOVING_WALL) a.moving_mask |= 1u << fc;
  }
  a.outlet_wave = outlet_wave_mask(c->geom, a.outlet_mask);
  const unsigned separate = a.outlet_mask & ~a.outlet_wave;
  const double* F = c->cfg.body_force;
  const int fgrid = (int)((c->face_stride + 255) / 256 < 4096 ? (c->face_stride + 255) / 256 : 4096);
  for (int fc = 0; fc < 6; ++fc) {
    if (!((separate >> fc) & 1u)) continue;
    k_outlet_velocity_canon<<<fgrid, 256, 0, c->stream>>>(c->geom, fc, f, F[0], F[1], F[2],
                                                          c->outlet_u, c->face_stride);
  }
  const size_t lds = c->np > 0 ? (sizeof(LdsEntry) + 9 * sizeof(double)) *
                                     (size_t)c->cfg.max_tile_particles
                               : 0;
  const bool walls = !(c->geom.periodic[0] && c->geom.periodic[1] && c->geom.periodic[2]);
  if (c->geom.q == 9) {
    if (walls) k_adjoint<9, true><<<c->ntiles, BLOCK, lds, c->stream>>>(a);
    else k_adjoint<9, false><<<c->ntiles, BLOCK, lds, c->stream>>>(a);
  } else {
    if (walls) k_adjoint<19, true><<<c->ntiles, BLOCK, lds, c->stream>>>(a);
    else k_adjoint<19, false><<<c->ntiles, BLOCK, lds, c->stream>>>(a);
  }
  int rc = hip_ok(hipGetLastError());
  if (rc) return rc;
  for (int fc = 0; fc < 6; ++fc) {
    if (!((separate >> fc) & 1u)) continue;
    if (c->geom.q == 9)
      k_outlet_adjoint<9><<<fgrid, 256, 0, c->stream>>>(c->geom, fc, f, c->outlet_g, lam_out,
                                                        F[0], F[1], F[2], c->face_stride);
    else
      k_outlet_adjoint<19><<<fgrid, 256, 0, c->stream>>>(c->geom, fc, f, c->outlet_g, lam_out,
                                                         F[0], F[1], F[2], c->face_stride);
  }
  return hip_ok(hipGetLastError());
}

int launch_rasterize_adjoint(psclbm_ctx* c, const double* gs, int kslots, double* gX) {
  const size_t lds = (sizeof(LdsEntry) + sizeof(double)) * (size_t)c->cfg.max_tile_particles;
  if (c->geom.q == 9)
    k_rasterize_adjoint<2><<<c->ntiles, BLOCK, lds, c->stream>>>(
        c->geom, c->cfg.shell_h, c->np, c->cfg.max_tile_particles, c->tile_count, c->tile_list,
        c->snap, gs, kslots, gX);
  else
    k_rasterize_adjoint<3><<<c->ntiles, BLOCK, lds, c->stream>>>(
        c->geom, c->cfg.shell_h, c->np, c->cfg.max_tile_particles, c->tile_count, c->tile_list,
        c->snap, gs, kslots, gX);
  return hip_ok(hipGetLastError());
}

}  // namespace psclbm
