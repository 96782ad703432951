// Per-cell arithmetic of the relativistic MRT lattice Boltzmann step (device).
//
// The state of a cell is its 19 f and 19 g populations stored as deviations
// from a rest reference state (n_r, P_r) of the member:
//   f_a = w_a n_r + f~_a,   g_a = gref_a + g~_a,
//   gref = (P_r, P_r/6 on the faces, P_r/12 on the edges) = g_eq(3 P_r, P_r, 0).
// Storing the deviation keeps FP32 rounding relative to the departure from the
// reference instead of to the full population; it costs one add per reference
// moment and nothing per population.
//
// Per cell (Sec. II and Sec. V.A of the paper):
//   1. Eq. (10) sums in FP64: N = sum f (= n gamma), E = sum g (= sigma - P),
//      M = sum e g (= sigma u).
//   2. Recovery in FP64 with P = eps/3: u = 3 M / (2E + sqrt(4E^2 - 3|M|^2)),
//      sigma = 4E / (3 + u^2), P = sigma (1 - u^2) / 4. A cell with E <= 0 or
//      |M| >= E is inadmissible: it is left uncollided and reported.
//   3. f: BGK, Eq. (5), with f_eq of Eq. (7) (n gamma = N).
//   4. g: MRT, Eqs. (30), (35), in the orthogonal D3Q19 moment basis
//      (rho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, 3pi_xx, p_ww, pi_ww,
//      p_xy, p_yz, p_xz, m_x, m_y, m_z). M has integer entries, so m = M g and
//      g* = g - M^-1 S (m - m_eq) are applied in factored form on the sums and
//      differences of opposite populations, with the entries of M as
//      instruction constants; M^-1 = M^T diag(1/|row|^2) (orthogonal rows).
//      m_eq is evaluated in closed form from sigma, P, u (it equals M g_eq of
//      Eqs. 8-9). The conserved rows (rho, j) keep m* = m (tau_sigma = tau_j = dt).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rlb {

// Relaxation rates 1/tau of one member (Eq. 31 generalised to D3Q19).
struct Rates {
  double w_f;    // 1/tau_f   (f, Eq. 5)
  double s_e;    // 1/tau_e   (e row)
  double s_eps;  // 1/tau_eps (eps row)
  double s_q;    // 1/tau_q   (q, 3pi_xx, pi_ww, m rows)
  double s_v;    // 1/tau_v   (3p_xx, p_ww, p_xy, p_yz, p_xz rows)
};

// Extensions of the model read only by the kernels built for them (EXT):
// relaxation times set per cell from eta/s (local_rates), and the equation of
// state P = (Gamma - 1)(eps - m n) (recover_general).
struct Ext {
  double eta_s;  // > 0: tau_v of each cell from eta/s (Rates are the fallback)
  double kappa;  // shear-viscosity transformation factor
  double dof;    // degeneracy d_G of n_eq = d_G T^3 / pi^2
  double a_f, a_e, a_eps, a_q;  // > 0: tau_x - 1/2 = a_x (tau_v - 1/2)
  double eos_gamma;             // Gamma (general_eos only)
  double mass;                  // rest mass m (general_eos only)
  int32_t q_tied;               // tau_q follows tau_v (tau_q <= 0 given)
  int32_t general_eos;          // 0: the paper's P = eps/3
};

// Rest reference state the populations are stored relative to.
struct Ref {
  double n;  // n_r
  double P;  // P_r
};

// Conservation sums of one cell, FP64: N, E, Mx, My, Mz.
struct Sums {
  double v[5];
};

// Velocity set (order of rlb.h).
__host__ __device__ constexpr int ex(int a) {
  constexpr int t[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  return t[a];
}
__host__ __device__ constexpr int ey(int a) {
  constexpr int t[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  return t[a];
}
__host__ __device__ constexpr int ez(int a) {
  constexpr int t[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  return t[a];
}
// Lattice weights 1/3, 1/18, 1/36 (rest, faces, edges).
__host__ __device__ constexpr double weight(int a) {
  return a == 0 ? 1.0 / 3.0 : (a < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}
// Reference g populations in units of P_r.
__host__ __device__ constexpr double gref_unit(int a) {
  return a == 0 ? 1.0 : (a < 7 ? 1.0 / 6.0 : 1.0 / 12.0);
}

// Squared norms of the basis rows (sum over the velocities of row^2).
constexpr double kNormE = 2394.0, kNormEps = 252.0, kNormQ = 40.0, kNorm3P = 36.0,
                 kNorm3Pi = 72.0, kNormW = 12.0, kNormWPi = 24.0, kNormPxy = 4.0, kNormM = 8.0;

// FP64 sums of the stored g values: gs = sum g~, E = 3 P_r + gs, M = sum e g~
// (the reference has no momentum).
template <typename C>
__device__ __forceinline__ void g_sums(const C (&g)[19], const Ref& ref, double& E, double& Mx,
                                       double& My, double& Mz, double& gs) {
  double gd[19];
#pragma unroll
  for (int a = 0; a < 19; ++a) gd[a] = (double)g[a];
  // opposite pairs (a, a+1) for a odd
  const double S1 = gd[1] + gd[2], S3 = gd[3] + gd[4], S5 = gd[5] + gd[6];
  const double S7 = gd[7] + gd[8], S9 = gd[9] + gd[10], S11 = gd[11] + gd[12];
  const double S13 = gd[13] + gd[14], S15 = gd[15] + gd[16], S17 = gd[17] + gd[18];
  const double D1 = gd[1] - gd[2], D3 = gd[3] - gd[4], D5 = gd[5] - gd[6];
  const double D7 = gd[7] - gd[8], D9 = gd[9] - gd[10], D11 = gd[11] - gd[12];
  const double D13 = gd[13] - gd[14], D15 = gd[15] - gd[16], D17 = gd[17] - gd[18];
  gs = gd[0] + ((S1 + S3) + (S5 + S7)) + ((S9 + S11) + (S13 + S15)) + S17;
  E = 3.0 * ref.P + gs;
  Mx = D1 + (D7 + D9) + (D11 + D13);
  My = D3 + (D7 - D9) + (D15 + D17);
  Mz = D5 + (D11 - D13) + (D15 - D17);
}

// FP64 Eq. (10) sums of a cell from its stored deviations. fs and gs are the
// plain sums of the stored f and g values (N = n_r + fs, E = 3 P_r + gs).
template <typename C>
__device__ __forceinline__ void cell_sums(const C (&f)[19], const C (&g)[19], const Ref& ref,
                                          double& N, double& E, double& Mx, double& My,
                                          double& Mz, double& fs, double& gs) {
  fs = 0.0;
#pragma unroll
  for (int a = 0; a < 19; ++a) fs += (double)f[a];
  N = ref.n + fs;
  g_sums(g, ref, E, Mx, My, Mz, gs);
}

// Recovery (FP64). Returns false for an inadmissible cell.
struct Macro {
  double ux, uy, uz, u2, sigma, P;
};

__device__ __forceinline__ bool recover(double E, double Mx, double My, double Mz, Macro& m) {
  const double M2 = Mx * Mx + My * My + Mz * Mz;
  const bool ok = (E > 0.0) && (M2 < E * E);
  const double Es = ok ? E : 1.0;
  const double M2s = ok ? M2 : 0.0;
  const double q = 3.0 / (2.0 * Es + sqrt(4.0 * Es * Es - 3.0 * M2s));
  m.ux = ok ? q * Mx : 0.0;
  m.uy = ok ? q * My : 0.0;
  m.uz = ok ? q * Mz : 0.0;
  m.u2 = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
  m.sigma = 4.0 * Es / (3.0 + m.u2);
  m.P = 0.25 * m.sigma * (1.0 - m.u2);
  return ok;
}

// Recovery for the equation of state P = (Gamma - 1)(eps - m n) (an extension;
// Gamma = 4/3, m = 0 is the paper's P = eps/3). With z = sigma = (eps + P) gamma^2,
// Eq. (10) gives z = E + P, u = M / z, eps + P = z - |M|^2/z, n = N / gamma:
//   F(z) = z - E - c [(z - |M|^2/z) - m N sqrt(1 - |M|^2/z^2)] = 0, c = (Gamma-1)/Gamma.
// F increases on (|M|, Gamma E] with F(|M|) < 0 <= F(Gamma E): Newton from the
// root at rest, kept inside the shrinking bracket (bisection when a step
// leaves it), FP64. A step at the rounding level ends the iteration before
// the bracket test: Newton approaching from one side leaves the other end of
// the bracket where it started, and such a step lands on the near end, so
// testing it first would throw z back to the middle of the initial bracket.
// A cell needs E > 0, |M| < E, N >= 0 and P > 0.
__device__ __forceinline__ bool recover_general(double N, double E, double Mx, double My,
                                                double Mz, const Ext& x, Macro& m) {
  const double G = x.eos_gamma, c = (x.eos_gamma - 1.0) / x.eos_gamma, mass = x.mass;
  const double M2 = Mx * Mx + My * My + Mz * Mz;
  const bool ok0 = (E > 0.0) && (M2 < E * E) && (N >= 0.0);
  const double Es = ok0 ? E : 1.0, M2s = ok0 ? M2 : 0.0, mN = ok0 ? mass * N : 0.0;
  double lo = sqrt(M2s), hi = G * Es;
  // start from the root at rest, z = Gamma E - (Gamma - 1) m N (exact for M = 0)
  double z = fmin(fmax(G * Es - (G - 1.0) * mN, lo), hi);
  // F is evaluated near double precision: 1/z from the hardware reciprocal plus
  // one Newton-Raphson refinement (which squares its relative error) and an
  // IEEE square root. The derivative only sets the step, so it uses the
  // unrefined reciprocal square root; the bracket keeps every step safe.
  double inv_z = 0.0;
  for (int it = 0; it < 64; ++it) {
    const double r = __builtin_amdgcn_rcp(z);
    inv_z = fma(fma(-z, r, 1.0), r, r);
    const double Mz_ = M2s * inv_z;
    const double x2 = Mz_ * inv_z;
    const double sq = sqrt(1.0 - x2);
    const double Fz = z - Es - c * ((z - Mz_) - mN * sq);
    if (Fz > 0.0)
      hi = z;
    else
      lo = z;
    const double dF = 1.0 - c * (1.0 + x2 - mN * x2 * inv_z * __builtin_amdgcn_rsq(1.0 - x2));
    double zn = z - Fz * __builtin_amdgcn_rcp(dF);
    const bool done = fabs(zn - z) <= 1e-15 * z;
    if (!done && !(zn > lo && zn < hi)) zn = 0.5 * (lo + hi);
    z = zn;
    if (done) break;
  }
  const double r = __builtin_amdgcn_rcp(z);
  inv_z = fma(fma(-z, r, 1.0), r, r);
  const double sq = sqrt(1.0 - M2s * inv_z * inv_z);
  const double P = c * ((z - M2s * inv_z) - mN * sq);
  const bool ok = ok0 && (P > 0.0);
  m.ux = ok ? Mx * inv_z : 0.0;
  m.uy = ok ? My * inv_z : 0.0;
  m.uz = ok ? Mz * inv_z : 0.0;
  m.u2 = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
  m.sigma = ok ? z : 4.0 / 3.0;
  m.P = ok ? P : 1.0 / 3.0;
  return ok;
}

// The recovery of the member's model.
__device__ __forceinline__ bool recover_model(double N, double E, double Mx, double My,
                                              double Mz, const Ext& x, Macro& m) {
  if (x.general_eos) return recover_general(N, E, Mx, My, Mz, x, m);
  return recover(E, Mx, My, Mz, m);
}

// Rates of one cell whose relaxation times follow from the ratio eta/s
// (Sec. III.B), from its particle number N = n gamma and recovered fields:
//   T = P / n (the ideal-gas relation n = P/T of the initial states),
//   n_eq = d_G T^3 / pi^2, lambda = n / n_eq, s = 4n - n ln(lambda),
//   eta = (eta/s) s, and the relation after Eq. (10) solved for tau:
//   tau_v = 1/2 + kappa eta / (c_s^2 (eps + P) gamma), (eps + P) gamma = sigma / gamma.
// tau_x (x = f, e, eps, q) with a_x > 0 follow as tau_x - 1/2 = a_x (tau_v - 1/2);
// tau_q also follows tau_v when tied. A cell with n <= 0 or P <= 0 keeps the
// member's fixed rates.
__device__ __forceinline__ Rates local_rates(const Rates& rt, const Ext& v, double N,
                                             const Macro& m) {
  constexpr double kPi = 3.141592653589793;
  const double gam = 1.0 / sqrt(1.0 - m.u2);
  const double n = N / gam;
  if (!(v.eta_s > 0.0) || !(n > 0.0) || !(m.P > 0.0)) return rt;
  const double T = m.P / n;
  const double n_eq = v.dof * T * T * T / (kPi * kPi);
  const double s = 4.0 * n - n * log(n / n_eq);
  const double eta = v.eta_s * s;
  const double tv = 0.5 + v.kappa * eta / ((1.0 / 3.0) * (m.sigma / gam));
  Rates r = rt;
  r.s_v = 1.0 / tv;
  if (v.q_tied) r.s_q = r.s_v;
  if (v.a_f > 0.0) r.w_f = 1.0 / (0.5 + v.a_f * (tv - 0.5));
  if (v.a_e > 0.0) r.s_e = 1.0 / (0.5 + v.a_e * (tv - 0.5));
  if (v.a_eps > 0.0) r.s_eps = 1.0 / (0.5 + v.a_eps * (tv - 0.5));
  if (v.a_q > 0.0) r.s_q = 1.0 / (0.5 + v.a_q * (tv - 0.5));
  return r;
}

// The 15 non-conserved moments of a population vector.
template <typename C>
struct NonConserved {
  C e, eps, qx, qy, qz, p3xx, pi3xx, pww, piww, pxy, pyz, pxz, mx, my, mz;
};

// m = M g on the non-conserved rows, from pair sums and differences.
template <typename C>
__device__ __forceinline__ NonConserved<C> moments_nc(const C (&g)[19]) {
  const C g0 = g[0];
  const C S1 = g[1] + g[2], S3 = g[3] + g[4], S5 = g[5] + g[6];
  const C S7 = g[7] + g[8], S9 = g[9] + g[10], S11 = g[11] + g[12];
  const C S13 = g[13] + g[14], S15 = g[15] + g[16], S17 = g[17] + g[18];
  const C D1 = g[1] - g[2], D3 = g[3] - g[4], D5 = g[5] - g[6];
  const C D7 = g[7] - g[8], D9 = g[9] - g[10], D11 = g[11] - g[12];
  const C D13 = g[13] - g[14], D15 = g[15] - g[16], D17 = g[17] - g[18];
  const C Sf = S1 + S3 + S5;
  const C Exy = S7 + S9, Exz = S11 + S13, Eyz = S15 + S17;
  const C Se = Exy + Exz + Eyz;
  const C xyz_p = Exy + Exz - C(2.0) * Eyz;
  NonConserved<C> m;
  m.e = C(-30.0) * g0 - C(11.0) * Sf + C(8.0) * Se;
  m.eps = C(12.0) * g0 - C(4.0) * Sf + Se;
  m.p3xx = C(2.0) * S1 - S3 - S5 + xyz_p;
  m.pi3xx = C(-4.0) * S1 + C(2.0) * S3 + C(2.0) * S5 + xyz_p;
  m.pww = S3 - S5 + Exy - Exz;
  m.piww = C(-2.0) * S3 + C(2.0) * S5 + Exy - Exz;
  m.pxy = S7 - S9;
  m.pxz = S11 - S13;
  m.pyz = S15 - S17;
  m.qx = C(-4.0) * D1 + D7 + D9 + D11 + D13;
  m.qy = C(-4.0) * D3 + D7 - D9 + D15 + D17;
  m.qz = C(-4.0) * D5 + D11 - D13 + D15 - D17;
  m.mx = D7 + D9 - D11 - D13;
  m.my = -D7 + D9 + D15 + D17;
  m.mz = D11 - D13 - D15 + D17;
  return m;
}

// g <- g - M^T c for a moment-space vector c (non-conserved rows only).
template <typename C>
__device__ __forceinline__ void sub_MT(C (&g)[19], const NonConserved<C>& c) {
  const C face = C(-11.0) * c.e - C(4.0) * c.eps;
  const C ev_x = face + C(2.0) * c.p3xx - C(4.0) * c.pi3xx;
  const C ev_y = face - c.p3xx + C(2.0) * c.pi3xx + c.pww - C(2.0) * c.piww;
  const C ev_z = face - c.p3xx + C(2.0) * c.pi3xx - c.pww + C(2.0) * c.piww;
  const C edge = C(8.0) * c.e + c.eps;
  const C ev_xy = edge + c.p3xx + c.pi3xx + c.pww + c.piww;
  const C ev_xz = edge + c.p3xx + c.pi3xx - c.pww - c.piww;
  const C ev_yz = edge - C(2.0) * (c.p3xx + c.pi3xx);
  const C od_x = C(-4.0) * c.qx, od_y = C(-4.0) * c.qy, od_z = C(-4.0) * c.qz;
  const C o7 = c.qx + c.qy + c.mx - c.my;
  const C o9 = c.qx - c.qy + c.mx + c.my;
  const C o11 = c.qx + c.qz - c.mx + c.mz;
  const C o13 = c.qx - c.qz - c.mx - c.mz;
  const C o15 = c.qy + c.qz + c.my - c.mz;
  const C o17 = c.qy - c.qz + c.my + c.mz;
  g[0] = g[0] - (C(-30.0) * c.e + C(12.0) * c.eps);
  g[1] = g[1] - (ev_x + od_x);
  g[2] = g[2] - (ev_x - od_x);
  g[3] = g[3] - (ev_y + od_y);
  g[4] = g[4] - (ev_y - od_y);
  g[5] = g[5] - (ev_z + od_z);
  g[6] = g[6] - (ev_z - od_z);
  g[7] = g[7] - (ev_xy + c.pxy + o7);
  g[8] = g[8] - (ev_xy + c.pxy - o7);
  g[9] = g[9] - (ev_xy - c.pxy + o9);
  g[10] = g[10] - (ev_xy - c.pxy - o9);
  g[11] = g[11] - (ev_xz + c.pxz + o11);
  g[12] = g[12] - (ev_xz + c.pxz - o11);
  g[13] = g[13] - (ev_xz - c.pxz + o13);
  g[14] = g[14] - (ev_xz - c.pxz - o13);
  g[15] = g[15] - (ev_yz + c.pyz + o15);
  g[16] = g[16] - (ev_yz + c.pyz - o15);
  g[17] = g[17] - (ev_yz - c.pyz + o17);
  g[18] = g[18] - (ev_yz - c.pyz - o17);
}

// m_eq on the non-conserved rows, minus the reference's moments, from the
// recovered fields (closed forms of M g_eq with g_eq of Eqs. 8-9).
template <typename C>
__device__ __forceinline__ NonConserved<C> equilibrium_nc(const Macro& mac, const Ref& ref) {
  const double sd = mac.sigma, Pd = mac.P, u2d = mac.u2;
  const C sg = (C)sd;
  const C ux = (C)mac.ux, uy = (C)mac.uy, uz = (C)mac.uz, uu = (C)u2d;
  const C sux = sg * ux, suy = sg * uy, suz = sg * uz;
  NonConserved<C> q;
  q.e = (C)(19.0 * sd * u2d + 87.0 * Pd - 30.0 * sd + 33.0 * ref.P);
  q.eps = (C)(12.0 * sd - 39.0 * Pd - 5.5 * sd * u2d - 9.0 * ref.P);
  q.qx = C(-2.0 / 3.0) * sux;
  q.qy = C(-2.0 / 3.0) * suy;
  q.qz = C(-2.0 / 3.0) * suz;
  q.p3xx = sg * (C(3.0) * ux * ux - uu);
  q.pi3xx = C(-0.5) * q.p3xx;
  q.pww = sg * (uy * uy - uz * uz);
  q.piww = C(-0.5) * q.pww;
  q.pxy = sux * uy;
  q.pxz = sux * uz;
  q.pyz = suy * uz;
  q.mx = q.my = q.mz = C(0.0);
  return q;
}

// c_k = s_k v_k / |row_k|^2.
template <typename C>
__device__ __forceinline__ NonConserved<C> scale_rates(const NonConserved<C>& v, const Rates& rt) {
  const C se = (C)rt.s_e, seps = (C)rt.s_eps, sq = (C)rt.s_q, sv = (C)rt.s_v;
  NonConserved<C> c;
  c.e = se * v.e * C(1.0 / kNormE);
  c.eps = seps * v.eps * C(1.0 / kNormEps);
  c.qx = sq * v.qx * C(1.0 / kNormQ);
  c.qy = sq * v.qy * C(1.0 / kNormQ);
  c.qz = sq * v.qz * C(1.0 / kNormQ);
  c.p3xx = sv * v.p3xx * C(1.0 / kNorm3P);
  c.pi3xx = sq * v.pi3xx * C(1.0 / kNorm3Pi);
  c.pww = sv * v.pww * C(1.0 / kNormW);
  c.piww = sq * v.piww * C(1.0 / kNormWPi);
  c.pxy = sv * v.pxy * C(1.0 / kNormPxy);
  c.pyz = sv * v.pyz * C(1.0 / kNormPxy);
  c.pxz = sv * v.pxz * C(1.0 / kNormPxy);
  c.mx = sq * v.mx * C(1.0 / kNormM);
  c.my = sq * v.my * C(1.0 / kNormM);
  c.mz = sq * v.mz * C(1.0 / kNormM);
  return c;
}

template <typename C>
__device__ __forceinline__ NonConserved<C> nc_sub(const NonConserved<C>& a,
                                                  const NonConserved<C>& b) {
  NonConserved<C> d;
  d.e = a.e - b.e;
  d.eps = a.eps - b.eps;
  d.qx = a.qx - b.qx;
  d.qy = a.qy - b.qy;
  d.qz = a.qz - b.qz;
  d.p3xx = a.p3xx - b.p3xx;
  d.pi3xx = a.pi3xx - b.pi3xx;
  d.pww = a.pww - b.pww;
  d.piww = a.piww - b.piww;
  d.pxy = a.pxy - b.pxy;
  d.pyz = a.pyz - b.pyz;
  d.pxz = a.pxz - b.pxz;
  d.mx = a.mx - b.mx;
  d.my = a.my - b.my;
  d.mz = a.mz - b.mz;
  return d;
}

// f: BGK, Eq. (5), in place. fs is the FP64 sum of the incoming stored f.
template <typename C>
__device__ __forceinline__ void collide_f(C (&f)[19], double N, double fs, const Macro& mac,
                                          const Rates& rt, const Ref& ref) {
  const C ux = (C)mac.ux, uy = (C)mac.uy, uz = (C)mac.uz, uu = (C)mac.u2;
  const C Nc = (C)N;
  const C b = (C)(N - ref.n) - C(1.5) * Nc * uu;  // deviation part of the w-bracket
  const C a3 = C(3.0) * Nc, a45 = C(4.5) * Nc;
  const C wf = (C)rt.w_f;
  const C w0 = C(1.0 / 3.0), w1 = C(1.0 / 18.0), w2 = C(1.0 / 36.0);
  C eu[19];
  eu[0] = C(0.0);
  eu[1] = ux;
  eu[2] = -ux;
  eu[3] = uy;
  eu[4] = -uy;
  eu[5] = uz;
  eu[6] = -uz;
  eu[7] = ux + uy;
  eu[8] = -(ux + uy);
  eu[9] = ux - uy;
  eu[10] = -(ux - uy);
  eu[11] = ux + uz;
  eu[12] = -(ux + uz);
  eu[13] = ux - uz;
  eu[14] = -(ux - uz);
  eu[15] = uy + uz;
  eu[16] = -(uy + uz);
  eu[17] = uy - uz;
  eu[18] = -(uy - uz);
#pragma unroll
  for (int a = 0; a < 19; ++a) {
    const C w = a == 0 ? w0 : (a < 7 ? w1 : w2);
    const C feq = w * (b + a3 * eu[a] + a45 * eu[a] * eu[a]);
    f[a] = f[a] + wf * (feq - f[a]);
  }
  // FP32 storage: the rounded outputs no longer sum to the incoming particle
  // number, and the residual is not zero on average (it builds up linearly
  // over steps). The rest population takes it back, computed in FP64.
  if constexpr (sizeof(C) == 4) {
    double fo = 0.0;
#pragma unroll
    for (int a = 1; a < 19; ++a) fo += (double)f[a];
    f[0] = (C)(fs - fo);
  }
}

// g: MRT, Eqs. (30), (35), in place. (E, M, gs) are the FP64 sums of the
// incoming stored g.
template <typename C>
__device__ __forceinline__ void collide_g(C (&g)[19], double Mx, double My, double Mz,
                                          double gs, const Macro& mac, const Rates& rt,
                                          const Ref& ref) {
  const NonConserved<C> m = moments_nc(g);
  const NonConserved<C> q = equilibrium_nc<C>(mac, ref);
  sub_MT(g, scale_rates(nc_sub(m, q), rt));
  // FP32 storage: as for f, the rounding residual of the conserved sums is
  // folded back in FP64: momentum into g_1, g_3, g_5 (one population per
  // axis), then energy into g_0 (the rest population carries no momentum).
  if constexpr (sizeof(C) == 4) {
    double gd[19];
#pragma unroll
    for (int a = 1; a < 19; ++a) gd[a] = (double)g[a];
    const double mx = (gd[1] - gd[2]) + ((gd[7] - gd[8]) + (gd[9] - gd[10])) +
                      ((gd[11] - gd[12]) + (gd[13] - gd[14]));
    const double my = (gd[3] - gd[4]) + ((gd[7] - gd[8]) - (gd[9] - gd[10])) +
                      ((gd[15] - gd[16]) + (gd[17] - gd[18]));
    const double mz = (gd[5] - gd[6]) + ((gd[11] - gd[12]) - (gd[13] - gd[14])) +
                      ((gd[15] - gd[16]) - (gd[17] - gd[18]));
    g[1] = (C)(gd[1] + (Mx - mx));
    g[3] = (C)(gd[3] + (My - my));
    g[5] = (C)(gd[5] + (Mz - mz));
    gd[1] = (double)g[1];
    gd[3] = (double)g[3];
    gd[5] = (double)g[5];
    double go = 0.0;
#pragma unroll
    for (int a = 1; a < 19; ++a) go += gd[a];
    g[0] = (C)(gs - go);
  }
}

// One collision of both distributions in place on the stored deviations.
// Returns admissibility; sums receives the FP64 Eq. (10) sums of the incoming
// populations. EXT: relaxation times of this cell from eta/s (local_rates).
template <typename C, bool EXT = false>
__device__ __forceinline__ bool collide(C (&f)[19], C (&g)[19], const Rates& rt, const Ref& ref,
                                        Sums& sums, const Ext* ext = nullptr) {
  double N, E, Mx, My, Mz, fs, gs;
  cell_sums(f, g, ref, N, E, Mx, My, Mz, fs, gs);
  sums.v[0] = N;
  sums.v[1] = E;
  sums.v[2] = Mx;
  sums.v[3] = My;
  sums.v[4] = Mz;
  Macro mac;
  if constexpr (EXT) {
    if (!recover_model(N, E, Mx, My, Mz, *ext, mac)) return false;
    const Rates r = local_rates(rt, *ext, N, mac);
    collide_f(f, N, fs, mac, r, ref);
    collide_g(g, Mx, My, Mz, gs, mac, r, ref);
  } else {
    if (!recover(E, Mx, My, Mz, mac)) return false;
    collide_f(f, N, fs, mac, rt, ref);
    collide_g(g, Mx, My, Mz, gs, mac, rt, ref);
  }
  return true;
}

// The g half alone (g never reads f): bit-identical to the g of collide().
template <typename C>
__device__ __forceinline__ bool collide_g_only(C (&g)[19], const Rates& rt, const Ref& ref) {
  double E, Mx, My, Mz, gs;
  g_sums(g, ref, E, Mx, My, Mz, gs);
  Macro mac;
  if (!recover(E, Mx, My, Mz, mac)) return false;
  collide_g(g, Mx, My, Mz, gs, mac, rt, ref);
  return true;
}

// Pressure of initial fields under the member's equation of state.
__device__ __forceinline__ double pressure_of(double eps, double n, const Ext& x) {
  if (x.general_eos) return (x.eos_gamma - 1.0) * (eps - x.mass * n);
  return eps / 3.0;
}

// Equilibrium deviations of a cell from its fields (init, Eqs. 7-9), FP64;
// P is the pressure of the fields (pressure_of).
__device__ __forceinline__ void equilibrium_dev(double n, double eps, double P, double ux,
                                                double uy, double uz, const Ref& ref,
                                                double (&f)[19], double (&g)[19]) {
  const double uu = ux * ux + uy * uy + uz * uz;
  const double gam2 = 1.0 / (1.0 - uu);
  const double N = n * sqrt(gam2);
  const double sigma = (eps + P) * gam2;
#pragma unroll
  for (int a = 0; a < 19; ++a) {
    const double eu = ex(a) * ux + ey(a) * uy + ez(a) * uz;
    const double w = weight(a);
    f[a] = w * (N * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu) - ref.n);
    double gv;
    if (a == 0)
      gv = w * (3.0 * sigma - 9.0 * P - 1.5 * sigma * uu);
    else
      gv = w * (3.0 * P + 3.0 * sigma * eu + 4.5 * sigma * eu * eu - 1.5 * sigma * uu);
    g[a] = gv - gref_unit(a) * ref.P;
  }
}

}  // namespace rlb
