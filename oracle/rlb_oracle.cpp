// FP64 CPU oracle for the relativistic lattice Boltzmann (RLB) model of
// Q. Li, K. H. Luo and X. J. Li, "Lattice Boltzmann method for relativistic
// hydrodynamics: issues on conservation law of particle number and
// discontinuities" (arXiv:1211.3286).
//
// TEST INFRASTRUCTURE ONLY. This library is loaded by the test-suite, by the
// package smoke check and by the CPU-baseline leg of the benchmark, and by
// nothing else. The GPU library shares no code, header, table or constant with
// it: the lattice, the moment basis and its inverse are built here on their own.
//
// What it computes, step by step in the paper's notation (all in double):
//   * D3Q19 velocities e_a, weights w_a, c_s^2 = 1/3, c = dx/dt = 1 (Sec. II).
//   * f_eq (Eq. 7), g_eq (Eqs. 8-9), moments n*gamma, sigma - P, sigma*u (Eq. 10).
//   * Recovery of (n, eps, P, gamma, u) from the three moments of Eq. (10)
//     with the equation of state P = eps/3, as the subluminal root of the
//     quadratic that Eq. (10) gives for |u|.
//   * f collision: BGK, Eq. (5).
//   * g collision: MRT, Eqs. (30), (31), (35): m = M g, m_eq = M g_eq,
//     m* = m - S (m - m_eq), g* = M^-1 m*, with tau_sigma = tau_j = dt for the
//     conserved rows. M is the orthogonal D3Q19 polynomial basis (the paper
//     prints only the D2Q9 case, Eq. 34); M^-1 is formed by Gauss-Jordan.
//   * Streaming: g(x + e_a, t + 1) = g*(x, t) (left side of Eqs. 5, 6, 35),
//     written as a pull with periodic wrap or zero-gradient clamp per axis.
//   * Adjoint of the g update (recovery, equilibria, MRT, streaming) by
//     complex-step Jacobians of the very same per-cell code.
//   * Extensions beyond the paper's runs: relaxation times per cell from
//     eta/s (cell_taus), and the equation of state P = (Gamma - 1)(eps - m n)
//     with its recovery by bisection (recover_general).
//   * The D2Q9 MRT model the paper itself runs (Sec. V.A, Eqs. 30-35): its
//     own velocity set, weights, basis (the rows that reproduce Eq. 34),
//     S of Eq. (31), g_eq of Eqs. (32)-(33), f_eq of Eq. (7)'s form with the
//     D2Q9 weights, the same recovery, on an nx x ny x 1 lattice.
//   * The correction term of Eqs. (37)-(38) on that model: C_7 of Eq. (38)
//     on the row-7 moment through (I - S/2) C, for flows along one axis (the
//     lattice's y, the paper's z), with central differences for the
//     derivatives. The printed sign belongs to the row e_flow^2 - e_perp^2;
//     this basis has row 7 = e_x^2 - e_y^2 with the flow along y, its
//     negative, so the term enters with a minus sign (a reading that a
//     Chapman-Enskog expansion of these equilibria confirms: only then does it
//     cancel the leading error of the row-7 flux; a test checks it).
//
// Readings where the paper is silent are listed in the design notes; each one
// used here is named at its place in the code.

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

typedef std::complex<double> cplx;

// ---------------------------------------------------------------------------
// Lattice (Sec. II, D3Q19). Ordering: rest, six faces, twelve edges; opposite
// directions are neighbours in the list. The weights are not printed in the
// paper: 1/3, 1/18, 1/36 are the D3Q19 weights with c_s^2 = 1/3.
// ---------------------------------------------------------------------------
const int EV[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

const double CS2 = 1.0 / 3.0;

double WV[19];
double MM[19][19];    // moment basis, row k = polynomial k evaluated at e_a
double MINV[19][19];  // its inverse
double NORM[19];      // squared row norms
bool tables_ready = false;

// Row polynomials of the orthogonal D3Q19 basis of d'Humieres et al. (2002):
// rho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, 3pi_xx, p_ww, pi_ww,
// p_xy, p_yz, p_xz, m_x, m_y, m_z.
double basis_poly(int k, double x, double y, double z) {
  double r2 = x * x + y * y + z * z;
  switch (k) {
    case 0: return 1.0;
    case 1: return 19.0 * r2 - 30.0;
    case 2: return (21.0 * r2 * r2 - 53.0 * r2 + 24.0) / 2.0;
    case 3: return x;
    case 4: return (5.0 * r2 - 9.0) * x;
    case 5: return y;
    case 6: return (5.0 * r2 - 9.0) * y;
    case 7: return z;
    case 8: return (5.0 * r2 - 9.0) * z;
    case 9: return 3.0 * x * x - r2;
    case 10: return (3.0 * r2 - 5.0) * (3.0 * x * x - r2);
    case 11: return y * y - z * z;
    case 12: return (3.0 * r2 - 5.0) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    case 18: return (x * x - y * y) * z;
  }
  return 0.0;
}

// Gauss-Jordan inverse with partial pivoting of an n x n row-major matrix.
void invert(int n, const double* A, double* Ainv) {
  std::vector<double> a(A, A + n * n);
  for (int i = 0; i < n * n; ++i) Ainv[i] = 0.0;
  for (int i = 0; i < n; ++i) Ainv[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[r * n + c]) > std::fabs(a[p * n + c])) p = r;
    if (p != c)
      for (int j = 0; j < n; ++j) {
        std::swap(a[p * n + j], a[c * n + j]);
        std::swap(Ainv[p * n + j], Ainv[c * n + j]);
      }
    double d = a[c * n + c];
    for (int j = 0; j < n; ++j) {
      a[c * n + j] /= d;
      Ainv[c * n + j] /= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = a[r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        a[r * n + j] -= f * a[c * n + j];
        Ainv[r * n + j] -= f * Ainv[c * n + j];
      }
    }
  }
}

void build_tables() {
  if (tables_ready) return;
  for (int a = 0; a < 19; ++a) {
    int r2 = EV[a][0] * EV[a][0] + EV[a][1] * EV[a][1] + EV[a][2] * EV[a][2];
    WV[a] = (r2 == 0) ? 1.0 / 3.0 : (r2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  for (int k = 0; k < 19; ++k) {
    NORM[k] = 0.0;
    for (int a = 0; a < 19; ++a) {
      MM[k][a] = basis_poly(k, EV[a][0], EV[a][1], EV[a][2]);
      NORM[k] += MM[k][a] * MM[k][a];
    }
  }
  invert(19, &MM[0][0], &MINV[0][0]);
  tables_ready = true;
}

// Rows of M that carry conserved quantities: rho (sigma - P) and j (sigma u).
inline bool conserved_row(int k) { return k == 0 || k == 3 || k == 5 || k == 7; }

// ---------------------------------------------------------------------------
// Parameters
// ---------------------------------------------------------------------------
struct Params {
  int32_t nx, ny, nz;
  int32_t bc[3];  // 0 periodic, 1 zero-gradient
  double tau_f, tau_v, tau_e, tau_eps, tau_q;
  // Relaxation times from eta/s per cell (off when eta_s <= 0), see cell_taus.
  double eta_s, kappa, dof, a_f, a_e, a_eps, a_q;
  // Equation of state P = (Gamma - 1)(eps - m n); Gamma = 0 or 4/3 with m = 0
  // is the paper's P = eps/3 (see recover_model).
  double eos_gamma, mass;
};

// Diagonal of S (Eq. 31 generalised to D3Q19). tau_sigma = tau_j = dt for the
// conserved rows (their deviation is set to zero, see collide_g). Reading: the
// D3Q19 ghost rows (q, 3pi_xx, pi_ww, m) all relax with tau_q, and tau_q <= 0
// means tau_q = tau_v (Case D of Sec. V.B sets tau_q = tau_v).
template <class T>
void rates(T tau_v, T tau_e, T tau_eps, T tau_q, T s[19]) {
  for (int k = 0; k < 19; ++k) s[k] = T(0.0);
  s[1] = T(1.0) / tau_e;
  s[2] = T(1.0) / tau_eps;
  s[4] = s[6] = s[8] = T(1.0) / tau_q;
  s[9] = s[11] = s[13] = s[14] = s[15] = T(1.0) / tau_v;
  s[10] = s[12] = T(1.0) / tau_q;
  s[16] = s[17] = s[18] = T(1.0) / tau_q;
}

inline double real_part(double v) { return v; }
inline double real_part(const cplx& v) { return v.real(); }

// ---------------------------------------------------------------------------
// Equilibria, Eqs. (7)-(9), with c_s^2 = 1/3 written out as in the paper.
// ---------------------------------------------------------------------------
template <class T>
void f_equilibrium(T n_gamma, const T u[3], T feq[19]) {
  T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int a = 0; a < 19; ++a) {
    T eu = T(EV[a][0]) * u[0] + T(EV[a][1]) * u[1] + T(EV[a][2]) * u[2];
    feq[a] = WV[a] * n_gamma *
             (T(1.0) + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

// sigma = (eps + P) gamma^2.
template <class T>
void g_equilibrium(T sigma, T P, const T u[3], T geq[19]) {
  T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  geq[0] = WV[0] * sigma * (T(3.0) - P * (2.0 + 3.0 * CS2) / (sigma * CS2) - uu / (2.0 * CS2));
  for (int a = 1; a < 19; ++a) {
    T eu = T(EV[a][0]) * u[0] + T(EV[a][1]) * u[1] + T(EV[a][2]) * u[2];
    geq[a] = WV[a] * sigma *
             (P / (sigma * CS2) + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

// ---------------------------------------------------------------------------
// Recovery of the fields from the moments of Eq. (10). With P = eps/3 and
// sigma = (eps + P) gamma^2 = 4 eps gamma^2 / 3, Eq. (10) reads
//   E = sigma - P = sigma (3 + u^2)/4,   M = sigma u,
// so |u| solves |M| u^2 - 4 E u + 3 |M| = 0. The subluminal root is
//   |u| = (2E - sqrt(4E^2 - 3|M|^2)) / |M| = 3|M| / (2E + sqrt(4E^2 - 3|M|^2)),
// and |u| < 1 exactly when |M| < E. A cell with E <= 0 or |M| >= E (or NaN)
// has no admissible state; it is reported and left uncollided (a reading).
// Squares are written as products so that complex-step derivatives stay exact.
// ---------------------------------------------------------------------------
template <class T>
struct Fields {
  T n, eps, P, gamma, u[3], sigma;
};

template <class T>
bool recover(T N, T E, const T M[3], Fields<T>& F) {
  T MM2 = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  double Er = real_part(E), M2r = real_part(MM2);
  if (!(Er > 0.0) || !(M2r < Er * Er)) return false;
  T q = T(3.0) / (T(2.0) * E + std::sqrt(T(4.0) * E * E - T(3.0) * MM2));
  for (int i = 0; i < 3; ++i) F.u[i] = q * M[i];
  T uu = F.u[0] * F.u[0] + F.u[1] * F.u[1] + F.u[2] * F.u[2];
  F.sigma = T(4.0) * E / (T(3.0) + uu);
  F.eps = T(0.75) * F.sigma * (T(1.0) - uu);
  F.P = F.eps / T(3.0);
  F.gamma = T(1.0) / std::sqrt(T(1.0) - uu);
  F.n = N / F.gamma;
  return true;
}

// ---------------------------------------------------------------------------
// Recovery for an equation of state other than the paper's (an extension):
// P = (Gamma - 1)(eps - m n), the gas with adiabatic index Gamma and rest mass
// m (m = 0, Gamma = 4/3 is P = eps/3). With z = sigma = (eps + P) gamma^2,
// Eq. (10) gives z = E + P, u = M / z, (eps + P) = z - |M|^2 / z,
// n = N / gamma, and so one equation in z:
//   F(z) = z - E - (Gamma - 1)/Gamma [ (z - |M|^2/z) - m N sqrt(1 - |M|^2/z^2) ] = 0.
// F is increasing, F(|M|) = |M| - E < 0 when |M| < E, and F(Gamma E) >= 0, so
// the root is unique in (|M|, Gamma E]; it is found here by plain bisection
// to the last bit. A cell needs E > 0, |M| < E, N >= 0 and P > 0 at the root.
// ---------------------------------------------------------------------------
bool general_eos(const Params& p) {
  return (p.eos_gamma != 0.0 && p.eos_gamma != 4.0 / 3.0) || p.mass != 0.0;
}

double eos_gamma_of(const Params& p) { return p.eos_gamma > 0.0 ? p.eos_gamma : 4.0 / 3.0; }

// Pressure of the initial fields under the member's equation of state.
double pressure_of(const Params& p, double eps, double n) {
  if (!general_eos(p)) return eps / 3.0;
  return (eos_gamma_of(p) - 1.0) * (eps - p.mass * n);
}

bool recover_general(const Params& p, double N, double E, const double M[3],
                     Fields<double>& F) {
  const double G = eos_gamma_of(p), m = p.mass;
  const double M2 = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  if (!(E > 0.0) || !(M2 < E * E) || !(N >= 0.0)) return false;
  auto pressure = [&](double z) {
    const double h = z - M2 / z;
    const double n = N * std::sqrt(1.0 - M2 / (z * z));
    return (G - 1.0) / G * (h - m * n);
  };
  double lo = std::sqrt(M2), hi = G * E;
  for (int i = 0; i < 4000; ++i) {
    const double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    if (mid - E - pressure(mid) > 0.0)
      hi = mid;
    else
      lo = mid;
  }
  const double z = 0.5 * (lo + hi);
  const double P = pressure(z);
  if (!(P > 0.0)) return false;
  for (int i = 0; i < 3; ++i) F.u[i] = M[i] / z;
  const double uu = F.u[0] * F.u[0] + F.u[1] * F.u[1] + F.u[2] * F.u[2];
  F.sigma = z;
  F.P = P;
  F.eps = (z - M2 / z) - P;
  F.gamma = 1.0 / std::sqrt(1.0 - uu);
  F.n = N / F.gamma;
  return true;
}

// The recovery of the member's model: the paper's closed form for P = eps/3,
// the bisection above otherwise.
bool recover_model(const Params& p, double N, double E, const double M[3], Fields<double>& F) {
  return general_eos(p) ? recover_general(p, N, E, M, F) : recover<double>(N, E, M, F);
}

template <class T>
void moments(const T f[19], const T g[19], T& N, T& E, T M[3]) {
  N = T(0.0);
  E = T(0.0);
  M[0] = M[1] = M[2] = T(0.0);
  for (int a = 0; a < 19; ++a) {
    N += f[a];
    E += g[a];
    for (int i = 0; i < 3; ++i) M[i] += T(EV[a][i]) * g[a];
  }
}

// g collision, Eqs. (30), (35): m = M g, m_eq = M g_eq,
// m* = m - S (m - m_eq), g* = M^-1 m*. Reading: the conserved rows relax with
// tau_sigma = tau_j = dt onto their own value, i.e. their (m - m_eq) is set to
// zero (it differs from zero only by the rounding of the recovery).
template <class T>
void collide_g(const T g[19], const Fields<T>& F, const T s[19], T gout[19]) {
  T geq[19], m[19], meq[19], ms[19];
  g_equilibrium(F.sigma, F.P, F.u, geq);
  for (int k = 0; k < 19; ++k) {
    m[k] = T(0.0);
    meq[k] = T(0.0);
    for (int a = 0; a < 19; ++a) {
      m[k] += MM[k][a] * g[a];
      meq[k] += MM[k][a] * geq[a];
    }
    T d = conserved_row(k) ? T(0.0) : (m[k] - meq[k]);
    ms[k] = m[k] - s[k] * d;
  }
  for (int a = 0; a < 19; ++a) {
    gout[a] = T(0.0);
    for (int k = 0; k < 19; ++k) gout[a] += MINV[a][k] * ms[k];
  }
}

// f collision, Eq. (5): f* = f - (f - f_eq) / tau_f.
template <class T>
void collide_f(const T f[19], const Fields<T>& F, double tau_f, T fout[19]) {
  T feq[19];
  f_equilibrium(F.n * F.gamma, F.u, feq);
  for (int a = 0; a < 19; ++a) fout[a] = f[a] - (f[a] - feq[a]) / tau_f;
}

// One cell of the g update from its pulled (pre-collision) populations.
// Returns false (and copies) when the cell is inadmissible.
template <class T>
bool cell_g(const T g[19], const T s[19], T gout[19]) {
  T E = T(0.0), M[3] = {T(0.0), T(0.0), T(0.0)};
  for (int a = 0; a < 19; ++a) {
    E += g[a];
    for (int i = 0; i < 3; ++i) M[i] += T(EV[a][i]) * g[a];
  }
  Fields<T> F;
  if (!recover(T(1.0), E, M, F)) {
    for (int a = 0; a < 19; ++a) gout[a] = g[a];
    return false;
  }
  collide_g(g, F, s, gout);
  return true;
}

// ---------------------------------------------------------------------------
// Streaming source: the cell that e_a points away from, per axis wrapped
// (periodic) or clamped (zero-gradient, the reading of "open" boundaries).
// ---------------------------------------------------------------------------
inline int src_coord(int c, int e, int N, int bc) {
  int s = c - e;
  if (bc == 0) {
    s %= N;
    if (s < 0) s += N;
  } else {
    if (s < 0) s = 0;
    if (s > N - 1) s = N - 1;
  }
  return s;
}

inline int64_t src_cell(const Params& p, int x, int y, int z, int a) {
  int sx = src_coord(x, EV[a][0], p.nx, p.bc[0]);
  int sy = src_coord(y, EV[a][1], p.ny, p.bc[1]);
  int sz = src_coord(z, EV[a][2], p.nz, p.bc[2]);
  return ((int64_t)sz * p.ny + sy) * p.nx + sx;
}

double tau_q_of(const Params& p) { return p.tau_q > 0.0 ? p.tau_q : p.tau_v; }

// ---------------------------------------------------------------------------
// Relaxation times of one cell. With eta_s > 0 they follow from the ratio of
// shear viscosity to entropy density, cell by cell (Sec. III.B):
//   T = P / n (the ideal-gas relation n = P/T of the initial states),
//   n_eq = d_G T^3 / pi^2, lambda = n / n_eq, s = 4n - n ln(lambda),
//   eta = (eta/s) s,
// and the viscosity relation after Eq. (10), eta = (tau - dt/2) c_s^2
// (eps + P) gamma, solved for tau, scaled by kappa (the transformation of the
// shear viscosity that Secs. IV and V.A call for; kappa = 1 is the plain
// relation): tau_v = 1/2 + kappa eta / (c_s^2 (eps + P) gamma).
// Each of tau_f, tau_e, tau_eps, tau_q with a_x > 0 follows as
// tau_x - 1/2 = a_x (tau_v - 1/2) (the parameterisation of the Cases of
// Sec. V.B); the others keep their fixed values. A cell with n <= 0 or P <= 0
// (no temperature) keeps the fixed values (a reading).
// ---------------------------------------------------------------------------
struct Taus {
  double f, v, e, eps, q;
};

Taus cell_taus(const Params& p, double n, double P, double gamma, double sigma) {
  Taus t{p.tau_f, p.tau_v, p.tau_e, p.tau_eps, tau_q_of(p)};
  if (!(p.eta_s > 0.0) || !(n > 0.0) || !(P > 0.0)) return t;
  const double T = P / n;
  const double n_eq = p.dof * T * T * T / (M_PI * M_PI);
  const double s_dens = 4.0 * n - n * std::log(n / n_eq);
  const double eta = p.eta_s * s_dens;
  const double eps_plus_P_gamma = sigma / gamma;  // (eps + P) gamma^2 / gamma
  t.v = 0.5 + p.kappa * eta / (CS2 * eps_plus_P_gamma);
  if (p.tau_q <= 0.0) t.q = t.v;
  if (p.a_f > 0.0) t.f = 0.5 + p.a_f * (t.v - 0.5);
  if (p.a_e > 0.0) t.e = 0.5 + p.a_e * (t.v - 0.5);
  if (p.a_eps > 0.0) t.eps = 0.5 + p.a_eps * (t.v - 0.5);
  if (p.a_q > 0.0) t.q = 0.5 + p.a_q * (t.v - 0.5);
  return t;
}

// ---------------------------------------------------------------------------
// D2Q9 lattice of Sec. V.A. Velocities: rest, (1,0), (0,1), (-1,0), (0,-1),
// (1,1), (-1,1), (-1,-1), (1,-1) in the (x, y) plane of an nx x ny x 1
// lattice; weights 4/9, 1/9, 1/36 (c_s^2 = 1/3). The moment basis is the
// orthogonal D2Q9 basis the paper takes from its Ref. [24]; restricted to
// g_eq of Eqs. (32)-(33) it gives the printed m_eq of Eq. (34), a property
// the tests check. Row order: rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy.
// ---------------------------------------------------------------------------
const int EV2[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                       {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
double WV2[9];
double MM2[9][9];
double MINV2[9][9];
bool tables2_ready = false;

double basis_poly2(int k, double x, double y) {
  double r2 = x * x + y * y;
  switch (k) {
    case 0: return 1.0;
    case 1: return 3.0 * r2 - 4.0;
    case 2: return (9.0 * r2 * r2 - 21.0 * r2 + 8.0) / 2.0;
    case 3: return x;
    case 4: return (3.0 * r2 - 5.0) * x;
    case 5: return y;
    case 6: return (3.0 * r2 - 5.0) * y;
    case 7: return x * x - y * y;
    case 8: return x * y;
  }
  return 0.0;
}

void build_tables2() {
  if (tables2_ready) return;
  for (int a = 0; a < 9; ++a) {
    int r2 = EV2[a][0] * EV2[a][0] + EV2[a][1] * EV2[a][1];
    WV2[a] = (r2 == 0) ? 4.0 / 9.0 : (r2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
    for (int k = 0; k < 9; ++k) MM2[k][a] = basis_poly2(k, EV2[a][0], EV2[a][1]);
  }
  invert(9, &MM2[0][0], &MINV2[0][0]);
  tables2_ready = true;
}

// Rows of the D2Q9 basis that carry conserved quantities: rho and j.
inline bool conserved_row2(int k) { return k == 0 || k == 3 || k == 5; }

// Diagonal of S, Eq. (31): (1/tau_sigma, 1/tau_e, 1/tau_eps, 1/tau_j, 1/tau_q,
// 1/tau_j, 1/tau_q, 1/tau_v, 1/tau_v). The conserved rows (tau_sigma = tau_j =
// dt) have their deviation set to zero in collide_g2, so their entry is not
// used; it is stored as 0. tau_q <= 0 means tau_q = tau_v.
void rates2(const Params& p, double s[9]) {
  const double tq = p.tau_q > 0.0 ? p.tau_q : p.tau_v;
  s[0] = s[3] = s[5] = 0.0;
  s[1] = 1.0 / p.tau_e;
  s[2] = 1.0 / p.tau_eps;
  s[4] = s[6] = 1.0 / tq;
  s[7] = s[8] = 1.0 / p.tau_v;
}

// f_eq with the form of Eq. (7) and the D2Q9 weights (reading: f lives on
// the same lattice as g and keeps its BGK collision, Eq. 5).
void f_equilibrium2(double n_gamma, const double u[2], double feq[9]) {
  double uu = u[0] * u[0] + u[1] * u[1];
  for (int a = 0; a < 9; ++a) {
    double eu = EV2[a][0] * u[0] + EV2[a][1] * u[1];
    feq[a] = WV2[a] * n_gamma *
             (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

// g_eq of Eqs. (32)-(33), sigma = (eps + P) gamma^2.
void g_equilibrium2(double sigma, double P, const double u[2], double geq[9]) {
  double uu = u[0] * u[0] + u[1] * u[1];
  geq[0] = WV2[0] * sigma *
           (9.0 / 4.0 - P * (5.0 + 9.0 * CS2) / (4.0 * sigma * CS2) - uu / (2.0 * CS2));
  for (int a = 1; a < 9; ++a) {
    double eu = EV2[a][0] * u[0] + EV2[a][1] * u[1];
    geq[a] = WV2[a] * sigma *
             (P / (sigma * CS2) + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

// Eq. (10) sums of a D2Q9 cell; M[2] = 0 (no z velocity).
void moments2(const double f[9], const double g[9], double& N, double& E, double M[3]) {
  N = E = 0.0;
  M[0] = M[1] = M[2] = 0.0;
  for (int a = 0; a < 9; ++a) {
    N += f[a];
    E += g[a];
    M[0] += EV2[a][0] * g[a];
    M[1] += EV2[a][1] * g[a];
  }
}

// One D2Q9 cell: recovery (same root as D3Q19, Eq. 10 with P = eps/3), f BGK
// (Eq. 5), g MRT (Eq. 35): m = M g, m_eq = M g_eq, m* = m - S (m - m_eq),
// g* = M^-1 m*. Returns false (and copies) when the cell is inadmissible.
bool cell2(const Params& p, const double s_fixed[9], const double f[9], const double g[9],
           double fout[9], double gout[9], double c7 = 0.0) {
  double N, E, M[3];
  moments2(f, g, N, E, M);
  Fields<double> F;
  if (!recover_model(p, N, E, M, F)) {
    for (int a = 0; a < 9; ++a) {
      fout[a] = f[a];
      gout[a] = g[a];
    }
    return false;
  }
  double s[9];
  double tau_f = p.tau_f;
  for (int k = 0; k < 9; ++k) s[k] = s_fixed[k];
  if (p.eta_s > 0.0) {  // relaxation times of this cell from eta/s
    const Taus t = cell_taus(p, F.n, F.P, F.gamma, F.sigma);
    Params q = p;
    q.tau_v = t.v;
    q.tau_e = t.e;
    q.tau_eps = t.eps;
    q.tau_q = t.q;
    rates2(q, s);
    tau_f = t.f;
  }
  double feq[9], geq[9], m[9], meq[9], ms[9];
  f_equilibrium2(F.n * F.gamma, F.u, feq);
  for (int a = 0; a < 9; ++a) fout[a] = f[a] - (f[a] - feq[a]) / tau_f;
  g_equilibrium2(F.sigma, F.P, F.u, geq);
  for (int k = 0; k < 9; ++k) {
    m[k] = meq[k] = 0.0;
    for (int a = 0; a < 9; ++a) {
      m[k] += MM2[k][a] * g[a];
      meq[k] += MM2[k][a] * geq[a];
    }
    double d = conserved_row2(k) ? 0.0 : (m[k] - meq[k]);
    ms[k] = m[k] - s[k] * d;
  }
  // Eq. (37): m* = m - S (m - m_eq) + (I - S/2) C with C = (0, ..., C_7, 0);
  // c7 is the correction of this basis' row 7 (see c7_row).
  ms[7] += (1.0 - 0.5 * s[7]) * c7;
  for (int a = 0; a < 9; ++a) {
    gout[a] = 0.0;
    for (int k = 0; k < 9; ++k) gout[a] += MINV2[a][k] * ms[k];
  }
  return true;
}

// Fields of a D2Q9 cell from its pre-collision g (Eq. 10 and the recovery).
bool fields2(const double g[9], Fields<double>& F) {
  double E = 0.0, M[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < 9; ++a) {
    E += g[a];
    M[0] += EV2[a][0] * g[a];
    M[1] += EV2[a][1] * g[a];
  }
  return recover<double>(1.0, E, M, F);
}

// C_7 as printed in Eq. (38) at a cell, the flow axis being y (the paper's
// z), dt = 1:
//   C_7 = 2 [u d(c_s^2 sigma - P) - c_s^2 sigma gamma^-1 u d(gamma)
//            - u d(sigma u^2) + u^2 theta d(sigma u)],
//   theta = 1 + 1 / ((eps/P + 1) gamma^2 - 1),
// u = u_y of the cell, d = the central difference (F(y+1) - F(y-1)) / 2 with
// the neighbours taken by the streaming rule of the y axis (wrap or clamp).
// Reading: C_7 = 0 when the cell or a neighbour is inadmissible.
double c7_term(const Fields<double>& F, bool ok, const Fields<double>& Fm, bool okm,
               const Fields<double>& Fp, bool okp) {
  if (!ok || !okm || !okp) return 0.0;
  auto x1 = [](const Fields<double>& G) { return CS2 * G.sigma - G.P; };
  auto su2 = [](const Fields<double>& G) { return G.sigma * G.u[1] * G.u[1]; };
  auto su = [](const Fields<double>& G) { return G.sigma * G.u[1]; };
  const double u = F.u[1];
  const double theta = 1.0 + 1.0 / ((F.eps / F.P + 1.0) * F.gamma * F.gamma - 1.0);
  const double d_x1 = 0.5 * (x1(Fp) - x1(Fm));
  const double d_gam = 0.5 * (Fp.gamma - Fm.gamma);
  const double d_su2 = 0.5 * (su2(Fp) - su2(Fm));
  const double d_su = 0.5 * (su(Fp) - su(Fm));
  return 2.0 * (u * d_x1 - CS2 * F.sigma / F.gamma * u * d_gam - u * d_su2 +
                u * u * theta * d_su);
}

// The correction of row 7 = e_x^2 - e_y^2 for a flow along y: the printed
// term belongs to the row e_flow^2 - e_perp^2 = -(row 7), hence the sign.
inline double c7_row(double c7_printed) { return -c7_printed; }

inline int64_t src_cell2(const Params& p, int x, int y, int a) {
  int sx = src_coord(x, EV2[a][0], p.nx, p.bc[0]);
  int sy = src_coord(y, EV2[a][1], p.ny, p.bc[1]);
  return (int64_t)sy * p.nx + sx;
}

int g_threads = 0;

}  // namespace

// ===========================================================================
// C entry points (ctypes). Populations are SoA: f[a * ncells + cell], the
// cell index is x + nx (y + ny z).
// ===========================================================================
extern "C" {

void oracle_set_threads(int n) {
  g_threads = n;
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#endif
}

int oracle_max_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_tables(int* e, double* w, double* M, double* Minv, double* norms) {
  build_tables();
  for (int a = 0; a < 19; ++a) {
    for (int i = 0; i < 3; ++i) e[a * 3 + i] = EV[a][i];
    w[a] = WV[a];
  }
  for (int k = 0; k < 19; ++k) {
    norms[k] = NORM[k];
    for (int a = 0; a < 19; ++a) {
      M[k * 19 + a] = MM[k][a];
      Minv[k * 19 + a] = MINV[k][a];
    }
  }
}

// D2Q9 velocities (9 x 2), weights and moment basis (row-major 9 x 9).
void oracle_d2q9_tables(int* e, double* w, double* M) {
  build_tables2();
  for (int a = 0; a < 9; ++a) {
    e[2 * a] = EV2[a][0];
    e[2 * a + 1] = EV2[a][1];
    w[a] = WV2[a];
    for (int k = 0; k < 9; ++k) M[k * 9 + a] = MM2[k][a];
  }
}

// D2Q9 g_eq, Eqs. (32)-(33); u has 2 components.
void oracle_d2q9_geq(double sigma, double P, const double* u, double* geq) {
  build_tables2();
  g_equilibrium2(sigma, P, u, geq);
}

// D2Q9 f_eq (Eq. 7's form, D2Q9 weights).
void oracle_d2q9_feq(double n, double gamma, const double* u, double* feq) {
  build_tables2();
  f_equilibrium2(n * gamma, u, feq);
}

void oracle_d2q9_rates(const Params* p, double* s) { rates2(*p, s); }

// Relaxation times {tau_f, tau_v, tau_e, tau_eps, tau_q} of a cell with fields
// (n, P, gamma, sigma) under the member's parameters (cell_taus).
void oracle_cell_taus(const Params* p, double n, double P, double gamma, double sigma,
                      double* out) {
  const Taus t = cell_taus(*p, n, P, gamma, sigma);
  out[0] = t.f;
  out[1] = t.v;
  out[2] = t.e;
  out[3] = t.eps;
  out[4] = t.q;
}

// Collision of one D2Q9 cell. Returns 1 if the cell was admissible.
int oracle_d2q9_collide_cell(const Params* p, const double* f, const double* g, double* fout,
                             double* gout) {
  build_tables2();
  double s[9];
  rates2(*p, s);
  return cell2(*p, s, f, g, fout, gout) ? 1 : 0;
}

// D2Q9 state at t = 0 on an nx x ny x 1 lattice: f = f_eq(n0, u0),
// g = g_eq(eps0, eps0/3, u0). u0 has 3 planes; the third must be zero.
void oracle_d2q9_init(const Params* p, const double* n0, const double* eps0, const double* u0,
                      double* f, double* g) {
  build_tables2();
  const int64_t nc = (int64_t)p->nx * p->ny;
  for (int64_t c = 0; c < nc; ++c) {
    double u[2] = {u0[c], u0[nc + c]};
    double uu = u[0] * u[0] + u[1] * u[1];
    double gamma = 1.0 / std::sqrt(1.0 - uu);
    double P = pressure_of(*p, eps0[c], n0[c]);
    double sigma = (eps0[c] + P) * gamma * gamma;
    double fe[9], ge[9];
    f_equilibrium2(n0[c] * gamma, u, fe);
    g_equilibrium2(sigma, P, u, ge);
    for (int a = 0; a < 9; ++a) {
      f[a * nc + c] = fe[a];
      g[a * nc + c] = ge[a];
    }
  }
}

// nsteps D2Q9 time steps in place: pull, sums, recovery, collisions; with
// correction != 0 the C_7 term of Eqs. (37)-(38) from the fields of the
// pulled state. Returns the number of inadmissible cell-updates.
int64_t oracle_d2q9_step(const Params* p, int32_t nsteps, double* f, double* g,
                         int32_t correction) {
  build_tables2();
  const int64_t nc = (int64_t)p->nx * p->ny;
  double s[9];
  rates2(*p, s);
  std::vector<double> fl((size_t)(9 * nc)), gl((size_t)(9 * nc));
  std::vector<Fields<double>> F((size_t)nc);
  std::vector<char> ok((size_t)nc);
  int64_t bad = 0;
  for (int t = 0; t < nsteps; ++t) {
    // streaming (pull) of every cell, then the fields of the pulled state
#pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        int64_t c = (int64_t)y * p->nx + x;
        double gc[9];
        for (int a = 0; a < 9; ++a) {
          int64_t sc = src_cell2(*p, x, y, a);
          fl[a * nc + c] = f[a * nc + sc];
          gl[a * nc + c] = gc[a] = g[a * nc + sc];
        }
        ok[c] = fields2(gc, F[c]);
      }
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        int64_t c = (int64_t)y * p->nx + x;
        double fc[9], gc[9], fo[9], go[9];
        for (int a = 0; a < 9; ++a) {
          fc[a] = fl[a * nc + c];
          gc[a] = gl[a * nc + c];
        }
        double c7 = 0.0;
        if (correction) {
          int64_t cm = (int64_t)src_coord(y, 1, p->ny, p->bc[1]) * p->nx + x;   // y - 1
          int64_t cp = (int64_t)src_coord(y, -1, p->ny, p->bc[1]) * p->nx + x;  // y + 1
          c7 = c7_row(c7_term(F[c], ok[c], F[cm], ok[cm], F[cp], ok[cp]));
        }
        if (!cell2(*p, s, fc, gc, fo, go, c7)) ++bad;
        for (int a = 0; a < 9; ++a) {
          f[a * nc + c] = fo[a];
          g[a * nc + c] = go[a];
        }
      }
  }
  return bad;
}

// Fields of a stored D2Q9 state (u has 3 planes, the third is 0) and the
// lattice sums {N, E, Mx, My, 0}. Returns the number of inadmissible cells.
int64_t oracle_d2q9_fields(const Params* p, const double* f, const double* g, double* n,
                           double* eps, double* P, double* gamma, double* u, double* sums) {
  build_tables2();
  const int64_t nc = (int64_t)p->nx * p->ny;
  int64_t bad = 0;
  double S[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t c = 0; c < nc; ++c) {
    double fl[9], gl[9];
    for (int a = 0; a < 9; ++a) {
      fl[a] = f[a * nc + c];
      gl[a] = g[a * nc + c];
    }
    double N, E, M[3];
    moments2(fl, gl, N, E, M);
    S[0] += N;
    S[1] += E;
    S[2] += M[0];
    S[3] += M[1];
    Fields<double> F;
    if (!recover_model(*p, N, E, M, F)) {
      ++bad;
      double q = std::nan("");
      F.n = F.eps = F.P = F.gamma = F.u[0] = F.u[1] = F.u[2] = q;
    }
    if (n) n[c] = F.n;
    if (eps) eps[c] = F.eps;
    if (P) P[c] = F.P;
    if (gamma) gamma[c] = F.gamma;
    if (u) {
      u[c] = F.u[0];
      u[nc + c] = F.u[1];
      u[2 * nc + c] = F.u[2];
    }
  }
  if (sums)
    for (int k = 0; k < 5; ++k) sums[k] = S[k];
  return bad;
}

void oracle_feq(double n, double gamma, const double* u, double* feq) {
  build_tables();
  f_equilibrium<double>(n * gamma, u, feq);
}

void oracle_geq(double eps, double P, const double* u, double* geq) {
  build_tables();
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double sigma = (eps + P) / (1.0 - uu);  // (eps + P) gamma^2
  g_equilibrium<double>(sigma, P, u, geq);
}

// out = {n, eps, P, gamma, ux, uy, uz, sigma}; returns 1 if admissible.
int oracle_recover(double N, double E, const double* M, double* out) {
  Fields<double> F;
  if (!recover<double>(N, E, M, F)) return 0;
  out[0] = F.n;
  out[1] = F.eps;
  out[2] = F.P;
  out[3] = F.gamma;
  out[4] = F.u[0];
  out[5] = F.u[1];
  out[6] = F.u[2];
  out[7] = F.sigma;
  return 1;
}

// Recovery under the member's equation of state (recover_model); out as in
// oracle_recover.
int oracle_recover_model(const Params* p, double N, double E, const double* M, double* out) {
  Fields<double> F;
  if (!recover_model(*p, N, E, M, F)) return 0;
  out[0] = F.n;
  out[1] = F.eps;
  out[2] = F.P;
  out[3] = F.gamma;
  out[4] = F.u[0];
  out[5] = F.u[1];
  out[6] = F.u[2];
  out[7] = F.sigma;
  return 1;
}

void oracle_rates(const Params* p, double* s) {
  rates<double>(p->tau_v, p->tau_e, p->tau_eps, tau_q_of(*p), s);
}

// Collision of one cell (pre-collision f, g -> post-collision). Returns 1 if
// the cell was admissible.
int oracle_collide_cell(const Params* p, const double* f, const double* g, double* fout,
                        double* gout) {
  build_tables();
  double N, E, M[3];
  moments<double>(f, g, N, E, M);
  Fields<double> F;
  if (!recover_model(*p, N, E, M, F)) {
    for (int a = 0; a < 19; ++a) {
      fout[a] = f[a];
      gout[a] = g[a];
    }
    return 0;
  }
  const Taus t = cell_taus(*p, F.n, F.P, F.gamma, F.sigma);
  double s[19];
  rates<double>(t.v, t.e, t.eps, t.q, s);
  collide_f<double>(f, F, t.f, fout);
  collide_g<double>(g, F, s, gout);
  return 1;
}

// State at t = 0: the equilibria of the initial fields (u has 3 planes),
// f = f_eq(n0, u0), g = g_eq(eps0, P0 = eps0/3, u0).
void oracle_init(const Params* p, const double* n0, const double* eps0, const double* u0,
                 double* f, double* g) {
  build_tables();
  const int64_t nc = (int64_t)p->nx * p->ny * p->nz;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nc; ++c) {
    double u[3] = {u0[c], u0[nc + c], u0[2 * nc + c]};
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double gamma = 1.0 / std::sqrt(1.0 - uu);
    double P = pressure_of(*p, eps0[c], n0[c]);
    double sigma = (eps0[c] + P) * gamma * gamma;
    double fe[19], ge[19];
    f_equilibrium<double>(n0[c] * gamma, u, fe);
    g_equilibrium<double>(sigma, P, u, ge);
    for (int a = 0; a < 19; ++a) {
      f[a * nc + c] = fe[a];
      g[a * nc + c] = ge[a];
    }
  }
}

// nsteps time steps in place. Each step: stream (pull), moments (Eq. 10),
// recovery, equilibria (Eqs. 7-9), f BGK (Eq. 5), g MRT (Eq. 35).
// Returns the number of inadmissible cell-updates.
int64_t oracle_step(const Params* p, int32_t nsteps, double* f, double* g) {
  build_tables();
  const int64_t nc = (int64_t)p->nx * p->ny * p->nz;
  double s[19];
  rates<double>(p->tau_v, p->tau_e, p->tau_eps, tau_q_of(*p), s);
  std::vector<double> fn((size_t)(19 * nc)), gn((size_t)(19 * nc));
  int64_t bad = 0;
  for (int t = 0; t < nsteps; ++t) {
#pragma omp parallel for schedule(static) reduction(+ : bad) collapse(2)
    for (int z = 0; z < p->nz; ++z)
      for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
          int64_t c = ((int64_t)z * p->ny + y) * p->nx + x;
          double fl[19], gl[19], fo[19], go[19];
          for (int a = 0; a < 19; ++a) {
            int64_t sc = src_cell(*p, x, y, z, a);
            fl[a] = f[a * nc + sc];
            gl[a] = g[a * nc + sc];
          }
          double N, E, M[3];
          moments<double>(fl, gl, N, E, M);
          Fields<double> F;
          if (!recover_model(*p, N, E, M, F)) {
            ++bad;
            for (int a = 0; a < 19; ++a) {
              fo[a] = fl[a];
              go[a] = gl[a];
            }
          } else if (p->eta_s > 0.0) {  // relaxation times of this cell from eta/s
            const Taus t = cell_taus(*p, F.n, F.P, F.gamma, F.sigma);
            double sl[19];
            rates<double>(t.v, t.e, t.eps, t.q, sl);
            collide_f<double>(fl, F, t.f, fo);
            collide_g<double>(gl, F, sl, go);
          } else {
            collide_f<double>(fl, F, p->tau_f, fo);
            collide_g<double>(gl, F, s, go);
          }
          for (int a = 0; a < 19; ++a) {
            fn[a * nc + c] = fo[a];
            gn[a * nc + c] = go[a];
          }
        }
    std::memcpy(f, fn.data(), sizeof(double) * 19 * nc);
    std::memcpy(g, gn.data(), sizeof(double) * 19 * nc);
  }
  return bad;
}

// Fields of a stored state plus the lattice sums of n*gamma, sigma - P and
// sigma*u (the T^{00}, T^{0i} integrals of Eqs. 2-3). Any output may be NULL.
// sums = {sum N, sum E, sum Mx, sum My, sum Mz}. Returns the number of
// inadmissible cells (their fields are NaN).
int64_t oracle_fields(const Params* p, const double* f, const double* g, double* n, double* eps,
                      double* P, double* gamma, double* u, double* sums) {
  build_tables();
  const int64_t nc = (int64_t)p->nx * p->ny * p->nz;
  int64_t bad = 0;
  double S0 = 0, S1 = 0, S2 = 0, S3 = 0, S4 = 0;
  for (int64_t c = 0; c < nc; ++c) {
    double fl[19], gl[19];
    for (int a = 0; a < 19; ++a) {
      fl[a] = f[a * nc + c];
      gl[a] = g[a * nc + c];
    }
    double N, E, M[3];
    moments<double>(fl, gl, N, E, M);
    S0 += N;
    S1 += E;
    S2 += M[0];
    S3 += M[1];
    S4 += M[2];
    Fields<double> F;
    bool ok = recover_model(*p, N, E, M, F);
    if (!ok) {
      ++bad;
      double q = std::nan("");
      F.n = F.eps = F.P = F.gamma = F.u[0] = F.u[1] = F.u[2] = q;
    }
    if (n) n[c] = F.n;
    if (eps) eps[c] = F.eps;
    if (P) P[c] = F.P;
    if (gamma) gamma[c] = F.gamma;
    if (u) {
      u[c] = F.u[0];
      u[nc + c] = F.u[1];
      u[2 * nc + c] = F.u[2];
    }
  }
  if (sums) {
    sums[0] = S0;
    sums[1] = S1;
    sums[2] = S2;
    sums[3] = S3;
    sums[4] = S4;
  }
  return bad;
}

// ---------------------------------------------------------------------------
// Adjoint of the g update (the loss involves only u and eps at the final time,
// and g never reads f, so f drops out).
//
// Forward: g*(0) = g_eq(eps0, eps0/3, u0); for t = 0..T-1,
//   g_pre(y) = g*(src(y, a), t), g*(y, t+1) = C(g_pre(y); tau).
// Loss gradient: dL/du(T), dL/deps(T) given per cell, with (u, eps) the
// recovery of g*(T).
// Reverse: gbar*(T) = (d(u,eps)/dg)^T (dL/du, dL/deps);
//   gbar_pre(y) = J_C(g_pre(y))^T gbar*(y, t+1),
//   dL/dtau_k += gbar*(y, t+1) . dC/dtau_k,
//   gbar*(x, t) = sum over (y, a) with src(y, a) = x of gbar_pre_a(y).
// Init: dL/deps0, dL/du0 = (d g_eq / d(eps0, u0))^T gbar*(0).
// Every Jacobian column is a complex-step derivative (h = 1e-30) of the same
// templated per-cell code the forward oracle runs: exact to rounding.
// tau is (tau_v, tau_e, tau_eps); tau_q follows tau_v when p->tau_q <= 0.
// ---------------------------------------------------------------------------
static const double CSH = 1e-30;

static void cell_g_real(const double g[19], const double s[19], double out[19]) {
  cell_g<double>(g, s, out);
}

static void rates_c(const Params& p, int which, cplx s[19]) {
  cplx tv(p.tau_v), te(p.tau_e), tpe(p.tau_eps);
  if (which == 0) tv += cplx(0.0, CSH);
  if (which == 1) te += cplx(0.0, CSH);
  if (which == 2) tpe += cplx(0.0, CSH);
  cplx tq = p.tau_q > 0.0 ? cplx(p.tau_q) : tv;
  rates<cplx>(tv, te, tpe, tq, s);
}

int oracle_grad(const Params* p, int32_t nsteps, const double* n0, const double* eps0,
                const double* u0, const double* dL_du, const double* dL_deps, double* dL_dtau,
                double* dL_deps0, double* dL_du0) {
  if (p->eta_s > 0.0 || general_eos(*p)) return -1;  // fixed taus, P = eps/3 only
  build_tables();
  (void)cell_g_real;
  const int64_t nc = (int64_t)p->nx * p->ny * p->nz;
  // Forward, storing g*(t) for t = 0..T.
  std::vector<double> tape((size_t)(nsteps + 1) * 19 * nc);
  std::vector<double> f((size_t)19 * nc);
  oracle_init(p, n0, eps0, u0, f.data(), tape.data());
  for (int t = 0; t < nsteps; ++t) {
    std::memcpy(tape.data() + (size_t)(t + 1) * 19 * nc, tape.data() + (size_t)t * 19 * nc,
                sizeof(double) * 19 * nc);
    oracle_step(p, 1, f.data(), tape.data() + (size_t)(t + 1) * 19 * nc);
  }
  double sr[19];
  rates<double>(p->tau_v, p->tau_e, p->tau_eps, tau_q_of(*p), sr);
  cplx sc[19];
  for (int k = 0; k < 19; ++k) sc[k] = cplx(sr[k]);
  cplx st[3][19];
  for (int w = 0; w < 3; ++w) rates_c(*p, w, st[w]);

  std::vector<double> gbar((size_t)19 * nc), gpre_bar((size_t)19 * nc);
  // Loss at T.
  const double* gT = tape.data() + (size_t)nsteps * 19 * nc;
  for (int64_t c = 0; c < nc; ++c) {
    for (int b = 0; b < 19; ++b) {
      cplx E(0.0), M[3] = {cplx(0.0), cplx(0.0), cplx(0.0)};
      for (int a = 0; a < 19; ++a) {
        cplx ga(gT[a * nc + c], a == b ? CSH : 0.0);
        E += ga;
        for (int i = 0; i < 3; ++i) M[i] += double(EV[a][i]) * ga;
      }
      Fields<cplx> F;
      double acc = 0.0;
      if (recover<cplx>(cplx(1.0), E, M, F)) {
        for (int i = 0; i < 3; ++i) acc += dL_du[i * nc + c] * F.u[i].imag() / CSH;
        acc += dL_deps[c] * F.eps.imag() / CSH;
      }
      gbar[b * nc + c] = acc;
    }
  }
  double dtau[3] = {0.0, 0.0, 0.0};
  for (int t = nsteps - 1; t >= 0; --t) {
    const double* gs = tape.data() + (size_t)t * 19 * nc;
    double dt0 = 0.0, dt1 = 0.0, dt2 = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : dt0, dt1, dt2) collapse(2)
    for (int z = 0; z < p->nz; ++z)
      for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
          int64_t c = ((int64_t)z * p->ny + y) * p->nx + x;
          double gl[19], ob[19];
          for (int a = 0; a < 19; ++a) {
            gl[a] = gs[a * nc + src_cell(*p, x, y, z, a)];
            ob[a] = gbar[a * nc + c];
          }
          cplx gc[19], out[19];
          for (int b = 0; b < 19; ++b) {
            for (int a = 0; a < 19; ++a) gc[a] = cplx(gl[a], a == b ? CSH : 0.0);
            cell_g<cplx>(gc, sc, out);
            double acc = 0.0;
            for (int a = 0; a < 19; ++a) acc += ob[a] * out[a].imag() / CSH;
            gpre_bar[b * nc + c] = acc;
          }
          double dtl[3];
          for (int w = 0; w < 3; ++w) {
            for (int a = 0; a < 19; ++a) gc[a] = cplx(gl[a], 0.0);
            cell_g<cplx>(gc, st[w], out);
            double acc = 0.0;
            for (int a = 0; a < 19; ++a) acc += ob[a] * out[a].imag() / CSH;
            dtl[w] = acc;
          }
          dt0 += dtl[0];
          dt1 += dtl[1];
          dt2 += dtl[2];
        }
    dtau[0] += dt0;
    dtau[1] += dt1;
    dtau[2] += dt2;
    // Transpose of the pull: scatter-add every pulled adjoint to its source.
    std::fill(gbar.begin(), gbar.end(), 0.0);
    for (int z = 0; z < p->nz; ++z)
      for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
          int64_t c = ((int64_t)z * p->ny + y) * p->nx + x;
          for (int a = 0; a < 19; ++a) gbar[a * nc + src_cell(*p, x, y, z, a)] +=
              gpre_bar[a * nc + c];
        }
  }
  dL_dtau[0] = dtau[0];
  dL_dtau[1] = dtau[1];
  dL_dtau[2] = dtau[2];
  // Init: g*(0) = g_eq(eps0, eps0/3, u0).
  for (int64_t c = 0; c < nc; ++c) {
    for (int w = 0; w < 4; ++w) {
      cplx e0(eps0[c], w == 0 ? CSH : 0.0);
      cplx u[3];
      for (int i = 0; i < 3; ++i) u[i] = cplx(u0[i * nc + c], w == i + 1 ? CSH : 0.0);
      cplx uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
      cplx P = e0 / 3.0;
      cplx sigma = (e0 + P) / (cplx(1.0) - uu);
      cplx ge[19];
      g_equilibrium<cplx>(sigma, P, u, ge);
      double acc = 0.0;
      for (int a = 0; a < 19; ++a) acc += gbar[a * nc + c] * ge[a].imag() / CSH;
      if (w == 0)
        dL_deps0[c] = acc;
      else
        dL_du0[(w - 1) * nc + c] = acc;
    }
  }
  return 0;
}

}  // extern "C"
