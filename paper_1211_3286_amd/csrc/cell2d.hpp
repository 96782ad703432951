// Per-cell arithmetic of the D2Q9 MRT model of Sec. V.A (device).
//
// The model the paper itself runs for its MRT study: Eqs. (30)-(35) on the
// D2Q9 lattice of an nx x ny x 1 lattice (x and y are the lattice axes).
// Velocities (order of rlb.h for RLB_D2Q9):
//   0 (0,0)  1 (1,0)  2 (0,1)  3 (-1,0)  4 (0,-1)
//   5 (1,1)  6 (-1,1)  7 (-1,-1)  8 (1,-1)
// opposite pairs (1,3), (2,4), (5,7), (6,8); weights 4/9, 1/9, 1/36.
//
// Storage, as for D3Q19: deviations from the member's rest reference state,
//   f_a = w_a n_r + f~_a,   g_a = gref_a + g~_a,
//   gref = (4/3 P_r, P_r/3 on the axes, P_r/12 on the diagonals)
//        = g_eq of Eqs. (32)-(33) at sigma = 4 P_r, P = P_r, u = 0.
//
// Moment basis (rows rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy; squared
// norms 9, 36, 36, 6, 12, 6, 12, 4, 4): the orthogonal D2Q9 basis that turns
// g_eq into the m_eq printed as Eq. (34):
//   e = -4 sigma + 3 sigma u^2 + 10 P,   eps = 4 sigma - 3 sigma u^2 - 13 P,
//   q = -sigma u,   p_xx = sigma (u_x^2 - u_y^2),   p_xy = sigma u_x u_y,
// and rho = sigma - P, j = sigma u (conserved: tau_sigma = tau_j = dt).
// S of Eq. (31): e <- 1/tau_e, eps <- 1/tau_eps, q <- 1/tau_q, p <- 1/tau_v.
// M has small integer entries, so m = M g and g* = g - M^T diag(1/|row|^2)
// S (m - m_eq) are written out on sums and differences of opposite pairs.
// The recovery is the D3Q19 one (Eq. 10 with P = eps/3) with M_z = 0, its two
// FP64 divisions taken as refined reciprocals (recover_xy).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cell.hpp"
#include "device_util.hpp"

namespace rlb {
namespace d2q9 {

__host__ __device__ constexpr int ex(int a) {
  constexpr int t[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  return t[a];
}
__host__ __device__ constexpr int ey(int a) {
  constexpr int t[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  return t[a];
}
__host__ __device__ constexpr double weight(int a) {
  return a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
}
// Reference g populations in units of P_r.
__host__ __device__ constexpr double gref_unit(int a) {
  return a == 0 ? 4.0 / 3.0 : (a < 5 ? 1.0 / 3.0 : 1.0 / 12.0);
}

constexpr double kNormE = 36.0, kNormEps = 36.0, kNormQ = 12.0, kNormP = 4.0;

// FP64 Eq. (10) sums from the stored deviations: N = n_r + fs, E = 3 P_r + gs,
// M = sum e g~ (the reference carries no momentum).
template <typename C>
__device__ __forceinline__ void cell_sums(const C (&f)[9], const C (&g)[9], const Ref& ref,
                                          double& N, double& E, double& Mx, double& My,
                                          double& fs, double& gs) {
  double gd[9];
  fs = 0.0;
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    fs += (double)f[a];
    gd[a] = (double)g[a];
  }
  const double D1 = gd[1] - gd[3], D2 = gd[2] - gd[4], D5 = gd[5] - gd[7], D6 = gd[6] - gd[8];
  gs = gd[0] + ((gd[1] + gd[3]) + (gd[2] + gd[4])) + ((gd[5] + gd[7]) + (gd[6] + gd[8]));
  N = ref.n + fs;
  E = 3.0 * ref.P + gs;
  Mx = D1 + (D5 - D6);
  My = D2 + (D5 + D6);
}

// The six non-conserved moments.
template <typename C>
struct NonConserved {
  C e, eps, qx, qy, pxx, pxy;
};

template <typename C>
__device__ __forceinline__ NonConserved<C> moments_nc(const C (&g)[9]) {
  const C S1 = g[1] + g[3], S2 = g[2] + g[4], S5 = g[5] + g[7], S6 = g[6] + g[8];
  const C D1 = g[1] - g[3], D2 = g[2] - g[4], D5 = g[5] - g[7], D6 = g[6] - g[8];
  const C Sa = S1 + S2, Sd = S5 + S6;
  NonConserved<C> m;
  m.e = C(-4.0) * g[0] - Sa + C(2.0) * Sd;
  m.eps = C(4.0) * g[0] - C(2.0) * Sa + Sd;
  m.qx = C(-2.0) * D1 + D5 - D6;
  m.qy = C(-2.0) * D2 + D5 + D6;
  m.pxx = S1 - S2;
  m.pxy = S5 - S6;
  return m;
}

// Eq. (34) on the non-conserved rows minus the reference's moments
// (e of gref = -6 P_r, eps of gref = 3 P_r).
template <typename C>
__device__ __forceinline__ NonConserved<C> equilibrium_nc(const Macro& mac, const Ref& ref) {
  const double sd = mac.sigma, Pd = mac.P, u2d = mac.u2;
  const C sg = (C)sd, ux = (C)mac.ux, uy = (C)mac.uy;
  NonConserved<C> q;
  q.e = (C)(-4.0 * sd + 3.0 * sd * u2d + 10.0 * Pd + 6.0 * ref.P);
  q.eps = (C)(4.0 * sd - 3.0 * sd * u2d - 13.0 * Pd - 3.0 * ref.P);
  q.qx = -(sg * ux);
  q.qy = -(sg * uy);
  q.pxx = sg * (ux * ux - uy * uy);
  q.pxy = sg * ux * uy;
  return q;
}

// c_k = s_k (m_k - m_eq,k) / |row_k|^2.
template <typename C>
__device__ __forceinline__ NonConserved<C> scaled_deviation(const NonConserved<C>& m,
                                                            const NonConserved<C>& q,
                                                            const Rates& rt) {
  const C se = (C)rt.s_e, seps = (C)rt.s_eps, sq = (C)rt.s_q, sv = (C)rt.s_v;
  NonConserved<C> c;
  c.e = se * (m.e - q.e) * C(1.0 / kNormE);
  c.eps = seps * (m.eps - q.eps) * C(1.0 / kNormEps);
  c.qx = sq * (m.qx - q.qx) * C(1.0 / kNormQ);
  c.qy = sq * (m.qy - q.qy) * C(1.0 / kNormQ);
  c.pxx = sv * (m.pxx - q.pxx) * C(1.0 / kNormP);
  c.pxy = sv * (m.pxy - q.pxy) * C(1.0 / kNormP);
  return c;
}

// g <- g - M^T c (non-conserved rows only).
template <typename C>
__device__ __forceinline__ void sub_MT(C (&g)[9], const NonConserved<C>& c) {
  const C axis = -c.e - C(2.0) * c.eps;
  const C diag = C(2.0) * c.e + c.eps;
  const C ax_x = axis + c.pxx, ax_y = axis - c.pxx;
  const C qx2 = C(2.0) * c.qx, qy2 = C(2.0) * c.qy;
  const C dp = diag + c.pxy, dm = diag - c.pxy;
  const C sp = c.qx + c.qy, sm = c.qx - c.qy;
  g[0] = g[0] - (C(-4.0) * c.e + C(4.0) * c.eps);
  g[1] = g[1] - (ax_x - qx2);
  g[3] = g[3] - (ax_x + qx2);
  g[2] = g[2] - (ax_y - qy2);
  g[4] = g[4] - (ax_y + qy2);
  g[5] = g[5] - (dp + sp);
  g[7] = g[7] - (dp - sp);
  g[6] = g[6] - (dm - sm);
  g[8] = g[8] - (dm + sm);
}

// f: BGK of Eq. (5) with f_eq of Eq. (7)'s form and the D2Q9 weights.
template <typename C>
__device__ __forceinline__ void collide_f(C (&f)[9], double N, double fs, const Macro& mac,
                                          const Rates& rt, const Ref& ref) {
  const C ux = (C)mac.ux, uy = (C)mac.uy, uu = (C)mac.u2;
  const C Nc = (C)N;
  const C b = (C)(N - ref.n) - C(1.5) * Nc * uu;
  const C a3 = C(3.0) * Nc, a45 = C(4.5) * Nc;
  const C wf = (C)rt.w_f;
  C eu[9];
  eu[0] = C(0.0);
  eu[1] = ux;
  eu[2] = uy;
  eu[3] = -ux;
  eu[4] = -uy;
  eu[5] = ux + uy;
  eu[6] = uy - ux;
  eu[7] = -(ux + uy);
  eu[8] = ux - uy;
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const C w = a == 0 ? C(4.0 / 9.0) : (a < 5 ? C(1.0 / 9.0) : C(1.0 / 36.0));
    const C feq = w * (b + a3 * eu[a] + a45 * eu[a] * eu[a]);
    f[a] = f[a] + wf * (feq - f[a]);
  }
  // FP32 storage: the rest population takes back the rounding residual of
  // the particle number, computed in FP64 (as for D3Q19).
  if constexpr (sizeof(C) == 4) {
    double fo = 0.0;
#pragma unroll
    for (int a = 1; a < 9; ++a) fo += (double)f[a];
    f[0] = (C)(fs - fo);
  }
}

// g: MRT of Eq. (35) in place; c7 is the correction of Eq. (37) on the
// p_xx row (0 without it): m*_7 gains (1 - s_v/2) c7.
template <typename C>
__device__ __forceinline__ void collide_g(C (&g)[9], double Mx, double My, double gs,
                                          const Macro& mac, const Rates& rt, const Ref& ref,
                                          double c7 = 0.0) {
  NonConserved<C> c = d2q9::scaled_deviation(d2q9::moments_nc(g),
                                             d2q9::equilibrium_nc<C>(mac, ref), rt);
  if (c7 != 0.0) c.pxx = c.pxx - (C)((1.0 - 0.5 * rt.s_v) * c7 * (1.0 / kNormP));
  d2q9::sub_MT(g, c);
  // FP32 storage: momentum residual into g_1 (x) and g_2 (y), then the
  // energy residual into the rest population, in FP64.
  if constexpr (sizeof(C) == 4) {
    double gd[9];
#pragma unroll
    for (int a = 1; a < 9; ++a) gd[a] = (double)g[a];
    const double mx = (gd[1] - gd[3]) + ((gd[5] - gd[7]) - (gd[6] - gd[8]));
    const double my = (gd[2] - gd[4]) + ((gd[5] - gd[7]) + (gd[6] - gd[8]));
    g[1] = (C)(gd[1] + (Mx - mx));
    g[2] = (C)(gd[2] + (My - my));
    gd[1] = (double)g[1];
    gd[2] = (double)g[2];
    double go = 0.0;
#pragma unroll
    for (int a = 1; a < 9; ++a) go += gd[a];
    g[0] = (C)(gs - go);
  }
}

// ---------------------------------------------------------------------------
// Correction term of Eqs. (37)-(38) for flows along y (the paper's z):
//   C_7 = 2 [u d(c_s^2 sigma - P) - c_s^2 sigma gamma^-1 u d(gamma)
//            - u d(sigma u^2) + u^2 theta d(sigma u)],
//   theta = 1 + 1 / ((eps/P + 1) gamma^2 - 1),
// u = u_y, d = central difference (F(y+1) - F(y-1)) / 2 over the neighbours
// the y-streaming rule picks (wrap or clamp), fields of the pulled state.
// The printed sign is that of the row e_flow^2 - e_perp^2; this basis' row 7
// is e_x^2 - e_y^2 = -(that row) for a flow along y, so it gets -C_7. A cell
// whose neighbour (or itself) is inadmissible gets no correction.
// ---------------------------------------------------------------------------
struct C7Fields {
  double x1, gam, su2, su;  // c_s^2 sigma - P, gamma, sigma u_y^2, sigma u_y
  bool ok;
};

__device__ __forceinline__ C7Fields c7_fields(const Macro& m, bool ok) {
  C7Fields F;
  F.ok = ok;
  F.x1 = m.sigma * (1.0 / 3.0) - m.P;
  F.gam = 1.0 / sqrt(1.0 - m.u2);
  F.su = m.sigma * m.uy;
  F.su2 = F.su * m.uy;
  return F;
}

// FP64 reciprocal: the hardware estimate refined by two Newton-Raphson steps
// (each squares the relative error), within an ulp or two of the IEEE
// quotient at a fraction of the instructions of a full division.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
}

// Eq. (10) with P = eps/3 in the plane: the subluminal root
// u = 3 M / (2E + sqrt(4E^2 - 3|M|^2)), sigma = 4E / (3 + u^2),
// P = sigma (1 - u^2) / 4; admissible iff E > 0 and |M| < E.
__device__ __forceinline__ bool recover_xy(double E, double Mx, double My, Macro& m) {
  const double M2 = Mx * Mx + My * My;
  const bool ok = (E > 0.0) && (M2 < E * E);
  const double Es = ok ? E : 1.0;
  const double M2s = ok ? M2 : 0.0;
  const double q = 3.0 * rcp_nr(2.0 * Es + sqrt(4.0 * Es * Es - 3.0 * M2s));
  m.ux = ok ? q * Mx : 0.0;
  m.uy = ok ? q * My : 0.0;
  m.uz = 0.0;
  m.u2 = m.ux * m.ux + m.uy * m.uy;
  m.sigma = 4.0 * Es * rcp_nr(3.0 + m.u2);
  m.P = 0.25 * m.sigma * (1.0 - m.u2);
  return ok;
}

// The recovery of the extended model in the plane: the general equation of
// state where one is set, else recover_xy (so that the per-cell rates and the
// fixed-rate kernels recover a cell alike, bit for bit).
__device__ __forceinline__ bool recover_model_xy(double N, double E, double Mx, double My,
                                                 const Ext& x, Macro& m) {
  if (x.general_eos) return recover_general(N, E, Mx, My, 0.0, x, m);
  return recover_xy(E, Mx, My, m);
}

// Fields of a cell from its pre-collision g (deviations from the reference).
__device__ __forceinline__ C7Fields c7_fields_of(const double (&gd)[9], const Ref& ref) {
  const double D1 = gd[1] - gd[3], D2 = gd[2] - gd[4], D5 = gd[5] - gd[7], D6 = gd[6] - gd[8];
  const double gs =
      gd[0] + ((gd[1] + gd[3]) + (gd[2] + gd[4])) + ((gd[5] + gd[7]) + (gd[6] + gd[8]));
  Macro m;
  const bool ok = recover_xy(3.0 * ref.P + gs, D1 + (D5 - D6), D2 + (D5 + D6), m);
  return c7_fields(m, ok);
}

// Fields of the cell whose pull offsets are off (its pre-collision g).
template <typename T>
__device__ __forceinline__ C7Fields c7_fields_at(const T* __restrict__ src, int64_t cs,
                                                 const uint32_t (&off)[9], const Ref& ref) {
  double gd[9];
#pragma unroll
  for (int a = 0; a < 9; ++a) gd[a] = (double)ld(src + (int64_t)(9 + a) * cs, off[a]);
  return c7_fields_of(gd, ref);
}

// Row-7 correction of a cell from its own recovery and its y-neighbours.
__device__ __forceinline__ double c7_row(const Macro& m, const C7Fields& fm,
                                         const C7Fields& fp) {
  if (!fm.ok || !fp.ok) return 0.0;
  const double u = m.uy;
  const double gam = 1.0 / sqrt(1.0 - m.u2);
  const double eps = 0.75 * m.sigma * (1.0 - m.u2);
  const double theta = 1.0 + 1.0 / ((eps / m.P + 1.0) * gam * gam - 1.0);
  const double d_x1 = 0.5 * (fp.x1 - fm.x1);
  const double d_gam = 0.5 * (fp.gam - fm.gam);
  const double d_su2 = 0.5 * (fp.su2 - fm.su2);
  const double d_su = 0.5 * (fp.su - fm.su);
  const double c7 = 2.0 * (u * d_x1 - (1.0 / 3.0) * m.sigma / gam * u * d_gam - u * d_su2 +
                           u * u * theta * d_su);
  return -c7;
}

// One collision of both distributions; false (cell untouched) if inadmissible.
// With CORR, fm / fp are the fields of the y - 1 and y + 1 neighbours and
// the correction of Eqs. (37)-(38) is applied. EXT: relaxation times of this
// cell from eta/s (local_rates).
// The collision in two stages: recovered() takes the sums of the pulled
// populations and the recovery, collide_recovered() the rest, so that a kernel
// can publish the cell's C_7 fields (c7_fields of the recovery) in between.
struct Recovered {
  double N, E, Mx, My, fs, gs;
  Macro mac;
  bool ok;
};

template <typename C, bool EXT = false>
__device__ __forceinline__ Recovered recovered(const C (&f)[9], const C (&g)[9], const Ref& ref,
                                               const Ext* ext = nullptr) {
  Recovered r;
  d2q9::cell_sums(f, g, ref, r.N, r.E, r.Mx, r.My, r.fs, r.gs);
  if constexpr (EXT)
    r.ok = recover_model_xy(r.N, r.E, r.Mx, r.My, *ext, r.mac);
  else
    r.ok = recover_xy(r.E, r.Mx, r.My, r.mac);
  return r;
}

template <typename C, bool CORR = false, bool EXT = false>
__device__ __forceinline__ bool collide_recovered(C (&f)[9], C (&g)[9], const Recovered& r,
                                                  const Rates& rt_member, const Ref& ref,
                                                  Sums& sums, const C7Fields* fm = nullptr,
                                                  const C7Fields* fp = nullptr,
                                                  const Ext* ext = nullptr) {
  sums.v[0] = r.N;
  sums.v[1] = r.E;
  sums.v[2] = r.Mx;
  sums.v[3] = r.My;
  sums.v[4] = 0.0;
  if (!r.ok) return false;
  Rates rt = rt_member;
  if constexpr (EXT) rt = local_rates(rt_member, *ext, r.N, r.mac);
  double c7 = 0.0;
  if constexpr (CORR) c7 = d2q9::c7_row(r.mac, *fm, *fp);
  d2q9::collide_f(f, r.N, r.fs, r.mac, rt, ref);
  d2q9::collide_g(g, r.Mx, r.My, r.gs, r.mac, rt, ref, c7);
  return true;
}

template <typename C, bool CORR = false, bool EXT = false>
__device__ __forceinline__ bool collide(C (&f)[9], C (&g)[9], const Rates& rt_member,
                                        const Ref& ref, Sums& sums,
                                        const C7Fields* fm = nullptr,
                                        const C7Fields* fp = nullptr,
                                        const Ext* ext = nullptr) {
  const Recovered r = recovered<C, EXT>(f, g, ref, ext);
  return collide_recovered<C, CORR, EXT>(f, g, r, rt_member, ref, sums, fm, fp, ext);
}

// Equilibrium deviations of a cell from its fields (Eqs. 7, 32, 33), FP64;
// P is the pressure of the fields.
__device__ __forceinline__ void equilibrium_dev(double n, double eps, double P, double ux,
                                                double uy, const Ref& ref, double (&f)[9],
                                                double (&g)[9]) {
  const double uu = ux * ux + uy * uy;
  const double gam2 = 1.0 / (1.0 - uu);
  const double N = n * sqrt(gam2);
  const double sigma = (eps + P) * gam2;
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const double eu = ex(a) * ux + ey(a) * uy;
    const double w = weight(a);
    f[a] = w * (N * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu) - ref.n);
    double gv;
    if (a == 0)
      gv = w * (2.25 * sigma - 6.0 * P - 1.5 * sigma * uu);
    else
      gv = w * (3.0 * P + 3.0 * sigma * eu + 4.5 * sigma * eu * eu - 1.5 * sigma * uu);
    g[a] = gv - gref_unit(a) * ref.P;
  }
}

// Byte offsets of the 9 pull sources of cell (x, y) (source = cell - e_a,
// clamped or wrapped per axis).
__device__ __forceinline__ void pull_offsets(int x, int y, int nx, int ny, int bcx, int bcy,
                                             uint32_t base, uint32_t esz, uint32_t (&off)[9],
                                             uint32_t& self) {
  const int xm = nbr(x, -1, nx, bcx), xp = nbr(x, 1, nx, bcx);
  const int ym = nbr(y, -1, ny, bcy), yp = nbr(y, 1, ny, bcy);
  const uint32_t unx = (uint32_t)nx;
  const uint32_t r_c = base + (uint32_t)y * unx;
  const uint32_t r_ym = base + (uint32_t)ym * unx;
  const uint32_t r_yp = base + (uint32_t)yp * unx;
  const uint32_t X = (uint32_t)x, XM = (uint32_t)xm, XP = (uint32_t)xp;
  off[0] = (r_c + X) * esz;
  off[1] = (r_c + XM) * esz;
  off[2] = (r_ym + X) * esz;
  off[3] = (r_c + XP) * esz;
  off[4] = (r_yp + X) * esz;
  off[5] = (r_ym + XM) * esz;
  off[6] = (r_ym + XP) * esz;
  off[7] = (r_yp + XP) * esz;
  off[8] = (r_yp + XM) * esz;
  self = off[0];
}

}  // namespace d2q9
}  // namespace rlb
