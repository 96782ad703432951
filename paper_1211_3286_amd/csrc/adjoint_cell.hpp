// Per-cell adjoint (reverse-mode derivative) of the g update of cell.hpp.
//
// Forward, per cell: g* = g - M^T c, c = S D^-1 (M g - m_eq(R(g))) on the
// non-conserved rows, D = diag(|row|^2), R the recovery (E, M) -> (sigma, P, u)
// and E = sum g, M = sum e g. Given gbar* = dL/dg*, the pre-collision adjoint is
//   gbar = gbar* - M^T lam + aE + e . aM,    lam = S D^-1 M gbar*,
// where (aE, aM) carries lam back through m_eq and R (only E and M depend on g
// through the recovery). The relaxation rates enter only through c, so
//   dL/dtau_k = (M gbar*)_k (m_k - m_eq,k) s_k^2 / |row_k|^2.
// The FP32 rounding fold-back of the forward is zero in exact arithmetic and
// is taken as the identity. Every derivative through the recovery and the
// equilibria is evaluated in FP64.
#pragma once

#include "cell.hpp"

namespace rlb {

// The recovery of cell.hpp with the intermediates its adjoint reuses:
// r = sqrt(4 E^2 - 3 |M|^2), q = 3 / (2E + r) (u = q M), and
// 1 / (3 + u^2) (sigma = 4 E / (3 + u^2)). Admissibility as in recover().
struct Recovered {
  Macro mac;
  double r, q, inv_den;
};

__device__ __forceinline__ bool recover_keep(double E, double Mx, double My, double Mz,
                                             Recovered& R) {
  const double M2 = Mx * Mx + My * My + Mz * Mz;
  const bool ok = (E > 0.0) && (M2 < E * E);
  const double Es = ok ? E : 1.0;
  const double M2s = ok ? M2 : 0.0;
  R.r = sqrt(4.0 * Es * Es - 3.0 * M2s);
  R.q = 3.0 / (2.0 * Es + R.r);
  Macro& m = R.mac;
  m.ux = ok ? R.q * Mx : 0.0;
  m.uy = ok ? R.q * My : 0.0;
  m.uz = ok ? R.q * Mz : 0.0;
  m.u2 = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
  R.inv_den = 1.0 / (3.0 + m.u2);
  m.sigma = 4.0 * Es * R.inv_den;
  m.P = 0.25 * m.sigma * (1.0 - m.u2);
  return ok;
}

// Adjoint of the recovery. In: the bars of sigma, P, u. Out: bars of E, M.
__device__ __forceinline__ void recovery_adjoint(double E, double Mx, double My, double Mz,
                                                 const Recovered& R, double sb, double Pb,
                                                 double ubx, double uby, double ubz, double& Eb,
                                                 double& Mbx, double& Mby, double& Mbz) {
  const Macro& mac = R.mac;
  // P = sigma (1 - u^2) / 4
  sb += 0.25 * (1.0 - mac.u2) * Pb;
  ubx -= 0.5 * mac.sigma * mac.ux * Pb;
  uby -= 0.5 * mac.sigma * mac.uy * Pb;
  ubz -= 0.5 * mac.sigma * mac.uz * Pb;
  // sigma = 4 E / (3 + u^2)
  Eb = 4.0 * sb * R.inv_den;
  const double t = -2.0 * mac.sigma * sb * R.inv_den;
  ubx += t * mac.ux;
  uby += t * mac.uy;
  ubz += t * mac.uz;
  // u = q M, q = 3 / D, D = 2E + r: dq/dD = -q^2 / 3, dr/dE = 4E / r, dr/dM = -3M / r
  const double q = R.q;
  Mbx = q * ubx;
  Mby = q * uby;
  Mbz = q * ubz;
  const double qb = ubx * Mx + uby * My + ubz * Mz;
  const double Db = -qb * q * q * (1.0 / 3.0);
  const double inv_r = 1.0 / R.r;
  Eb += 2.0 * Db + Db * 4.0 * E * inv_r;
  const double rm = -3.0 * Db * inv_r;
  Mbx += rm * Mx;
  Mby += rm * My;
  Mbz += rm * Mz;
}

// Adjoint of the closed-form m_eq (non-conserved rows): lam -> bars of sigma,
// P, u (added to sb, Pb, ub).
template <typename C>
__device__ __forceinline__ void equilibrium_adjoint(const NonConserved<C>& l, const Macro& mac,
                                                    double& sb, double& Pb, double& ubx,
                                                    double& uby, double& ubz) {
  const double ux = mac.ux, uy = mac.uy, uz = mac.uz, uu = mac.u2, s = mac.sigma;
  const double le = l.e, leps = l.eps, lqx = l.qx, lqy = l.qy, lqz = l.qz;
  const double lp = (double)l.p3xx - 0.5 * (double)l.pi3xx;  // 3p_xx and 3pi_xx share a form
  const double lw = (double)l.pww - 0.5 * (double)l.piww;    // p_ww and pi_ww likewise
  const double lxy = l.pxy, lyz = l.pyz, lxz = l.pxz;
  const double A = 3.0 * ux * ux - uu, B = uy * uy - uz * uz;
  sb += le * (19.0 * uu - 30.0) + leps * (12.0 - 5.5 * uu) -
        (2.0 / 3.0) * (lqx * ux + lqy * uy + lqz * uz) + lp * A + lw * B + lxy * ux * uy +
        lyz * uy * uz + lxz * ux * uz;
  Pb += 87.0 * le - 39.0 * leps;
  const double K = s * (19.0 * le - 5.5 * leps);
  const double sp = s * lp, sw = s * lw;
  ubx += 2.0 * K * ux - (2.0 / 3.0) * s * lqx + 4.0 * sp * ux + s * (lxy * uy + lxz * uz);
  uby += 2.0 * K * uy - (2.0 / 3.0) * s * lqy - 2.0 * sp * uy + 2.0 * sw * uy +
         s * (lxy * ux + lyz * uz);
  ubz += 2.0 * K * uz - (2.0 / 3.0) * s * lqz - 2.0 * sp * uz - 2.0 * sw * uz +
         s * (lyz * uy + lxz * ux);
}

// gbar[a] += aE + e_a . aM, in the precision of the adjoint populations (the
// four terms are rounded to it first).
template <typename C>
__device__ __forceinline__ void add_scalar_vector(C (&gb)[19], double aE, double ax, double ay,
                                                  double az) {
  const C e0 = (C)aE, cx = (C)ax, cy = (C)ay, cz = (C)az;
#pragma unroll
  for (int a = 0; a < 19; ++a)
    gb[a] = gb[a] + (e0 + C(ex(a)) * cx + C(ey(a)) * cy + C(ez(a)) * cz);
}

// Reverse of one g collision, in two phases so that the step kernel can read
// the forward populations of several cells before their adjoints. g: the
// cell's stored pre-collision populations; adjoint_prepare keeps what the
// reverse needs of them (sums, recovery, the non-equilibrium moments d).
template <typename C>
struct AdjPrep {
  double E, Mx, My, Mz;
  Recovered rec;
  NonConserved<C> d;
  bool ok;
};

template <typename C>
__device__ __forceinline__ void adjoint_prepare(const C (&g)[19], const Ref& ref, AdjPrep<C>& p) {
  double gs;
  g_sums(g, ref, p.E, p.Mx, p.My, p.Mz, gs);
  p.ok = recover_keep(p.E, p.Mx, p.My, p.Mz, p.rec);
  p.d = nc_sub(moments_nc(g), equilibrium_nc<C>(p.rec.mac, ref));
}

// gb: in gbar*, out gbar (pre-collision). dtau accumulates dL/dtau for the
// rate groups (v, e, eps, q). An inadmissible cell was not collided: identity.
template <typename C>
__device__ __forceinline__ void adjoint_apply(const AdjPrep<C>& p, C (&gb)[19], const Rates& rt,
                                              double (&dtau)[4]) {
  if (!p.ok) return;
  const NonConserved<C>& d = p.d;
  const NonConserved<C> mb = moments_nc(gb);
  const NonConserved<C> lam = scale_rates(mb, rt);
  // dL/dtau_k = mb_k d_k s_k^2 / |row_k|^2 (the 1 / |row|^2 folded into
  // constants: multiplications instead of FP64 divisions per cell and step)
  constexpr double i3P = 1.0 / kNorm3P, iW = 1.0 / kNormW, iPxy = 1.0 / kNormPxy,
                   iE = 1.0 / kNormE, iEps = 1.0 / kNormEps, iQ = 1.0 / kNormQ,
                   i3Pi = 1.0 / kNorm3Pi, iWPi = 1.0 / kNormWPi, iM = 1.0 / kNormM;
  const double sv2 = rt.s_v * rt.s_v, se2 = rt.s_e * rt.s_e, sp2 = rt.s_eps * rt.s_eps,
               sq2 = rt.s_q * rt.s_q;
  dtau[0] += sv2 * ((double)mb.p3xx * (double)d.p3xx * i3P +
                    (double)mb.pww * (double)d.pww * iW +
                    ((double)mb.pxy * (double)d.pxy + (double)mb.pyz * (double)d.pyz +
                     (double)mb.pxz * (double)d.pxz) * iPxy);
  dtau[1] += se2 * (double)mb.e * (double)d.e * iE;
  dtau[2] += sp2 * (double)mb.eps * (double)d.eps * iEps;
  dtau[3] += sq2 * (((double)mb.qx * (double)d.qx + (double)mb.qy * (double)d.qy +
                     (double)mb.qz * (double)d.qz) * iQ +
                    (double)mb.pi3xx * (double)d.pi3xx * i3Pi +
                    (double)mb.piww * (double)d.piww * iWPi +
                    ((double)mb.mx * (double)d.mx + (double)mb.my * (double)d.my +
                     (double)mb.mz * (double)d.mz) * iM);
  double sb = 0.0, Pb = 0.0, ubx = 0.0, uby = 0.0, ubz = 0.0;
  equilibrium_adjoint(lam, p.rec.mac, sb, Pb, ubx, uby, ubz);
  double aE, ax, ay, az;
  recovery_adjoint(p.E, p.Mx, p.My, p.Mz, p.rec, sb, Pb, ubx, uby, ubz, aE, ax, ay, az);
  sub_MT(gb, lam);
  add_scalar_vector(gb, aE, ax, ay, az);
}

// Adjoint of the fields read out at the end: (u, eps) of a stored state given
// dL/du and dL/deps. gb receives dL/dg* of that state.
template <typename C>
__device__ __forceinline__ void loss_adjoint(const C (&g)[19], const Ref& ref, double dux,
                                             double duy, double duz, double deps,
                                             C (&gb)[19]) {
  double E, Mx, My, Mz, gs;
  g_sums(g, ref, E, Mx, My, Mz, gs);
  Recovered R;
#pragma unroll
  for (int a = 0; a < 19; ++a) gb[a] = C(0.0);
  if (!recover_keep(E, Mx, My, Mz, R)) return;
  const Macro& mac = R.mac;
  // eps = (3/4) sigma (1 - u^2)
  const double sb = 0.75 * (1.0 - mac.u2) * deps;
  const double ubx = dux - 1.5 * mac.sigma * mac.ux * deps;
  const double uby = duy - 1.5 * mac.sigma * mac.uy * deps;
  const double ubz = duz - 1.5 * mac.sigma * mac.uz * deps;
  double aE, ax, ay, az;
  recovery_adjoint(E, Mx, My, Mz, R, sb, 0.0, ubx, uby, ubz, aE, ax, ay, az);
  add_scalar_vector(gb, aE, ax, ay, az);
}

// Adjoint of the initial state g* = g_eq(eps0, eps0/3, u0) (Eqs. 8-9).
template <typename C>
__device__ __forceinline__ void init_adjoint(const C (&gb)[19], double eps0, double ux,
                                             double uy, double uz, double& deps0, double& dux,
                                             double& duy, double& duz) {
  const double uu = ux * ux + uy * uy + uz * uz;
  const double gam2 = 1.0 / (1.0 - uu);
  const double P = eps0 / 3.0;
  const double s = (eps0 + P) * gam2;
  double sb = 0.0, Pb = 0.0, bx = 0.0, by = 0.0, bz = 0.0;
#pragma unroll
  for (int a = 0; a < 19; ++a) {
    const double b = (double)gb[a];
    const double w = weight(a);
    const double eu = ex(a) * ux + ey(a) * uy + ez(a) * uz;
    if (a == 0) {
      sb += b * w * (3.0 - 1.5 * uu);
      Pb += b * w * (-9.0);
      bx += b * w * (-3.0 * s * ux);
      by += b * w * (-3.0 * s * uy);
      bz += b * w * (-3.0 * s * uz);
    } else {
      sb += b * w * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
      Pb += b * w * 3.0;
      const double k = 3.0 * s + 9.0 * s * eu;
      bx += b * w * (k * ex(a) - 3.0 * s * ux);
      by += b * w * (k * ey(a) - 3.0 * s * uy);
      bz += b * w * (k * ez(a) - 3.0 * s * uz);
    }
  }
  // sigma = (4/3) eps0 / (1 - u^2), P = eps0 / 3
  deps0 = sb * (4.0 / 3.0) * gam2 + Pb / 3.0;
  const double t = sb * (4.0 / 3.0) * eps0 * 2.0 * gam2 * gam2;
  dux = bx + t * ux;
  duy = by + t * uy;
  duz = bz + t * uz;
}

}  // namespace rlb
