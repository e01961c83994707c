// Oracle (test infrastructure only): plain CPU FP64 reference implementation.
//
// Everything here follows the paper's definitions term by term, with no
// blocking, fusion or reordering: Section 2.1 (the reacting Navier-Stokes
// system, viscous stress, mixture-model species flux with the correction
// velocity), Section 2.2 (eighth-order centred first derivative and the
// eighth-order narrow variable-coefficient second-derivative stencil, eqs.
// for the flux-difference form and the face sum H with the 8x8 matrix M),
// Section 2.4 (chain rule for the correction-velocity terms).  Readings where
// the paper is silent (thermodynamic fits, rate law, transport model, form
// of the mixed viscous terms) are restated at each function.
//
// The right-hand side is evaluated one output cell at a time from primitive
// fields stored on the 4-layer periodic ghost grid; every derivative is taken
// from its nine samples along a grid line through the point.
#include "oracle.h"

#include <cmath>
#include <cstring>
#include <vector>
#include <omp.h>

#include "dual.hpp"

namespace {

const double RU = 8.31446261815324;   // J/(mol K)
const double PREF = 101325.0;         // Pa, standard-state pressure of K_p
const int NG = 4;                     // ghost layers

// ---------------------------------------------------------------- stencils
// Eighth-order centred first derivative (standard coefficients).
const double D1C[4] = {4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};

template <class S>
S d1(const S *f, double dx) {
  S r = 0.0;
  for (int s = 1; s <= 4; ++s) r = r + D1C[s - 1] * (f[4 + s] - f[4 - s]);
  return r / dx;
}

// The matrix M of the eighth-order narrow stencil, written out row by row as
// printed in Section 2.2 (rows 1..8 <-> m = -3..4, columns 1..8 <-> n = -3..4).
void narrow8(double m47, double m48, double M[8][8]) {
  const double m11 = 5.0 / 336.0 + m48;
  const double m12 = -83.0 / 3600.0 - m47 / 5.0 - 14.0 * m48 / 5.0;
  const double m13 = 299.0 / 50400.0 + 2.0 * m47 / 5.0 + 13.0 * m48 / 5.0;
  const double m14 = 17.0 / 12600.0 - m47 / 5.0 - 4.0 * m48 / 5.0;
  const double m15 = 1.0 / 1120.0;
  const double m21 = -11.0 / 560.0 - 2.0 * m48;
  const double m22 = -31.0 / 360.0 + m47 + 3.0 * m48;
  const double m23 = 41.0 / 200.0 - 9.0 * m47 / 5.0 + 4.0 * m48 / 5.0;
  const double m24 = -5927.0 / 50400.0 + 4.0 * m47 / 5.0 - 9.0 * m48 / 5.0;
  const double m25 = 17.0 / 600.0 - m47 / 5.0 - 4.0 * m48 / 5.0;
  const double m26 = -503.0 / 50400.0 + m47 / 5.0 + 4.0 * m48 / 5.0;
  const double m31 = -1.0 / 280.0;
  const double m32 = 1097.0 / 5040.0 - 2.0 * m47 + 6.0 * m48;
  const double m33 = -1349.0 / 10080.0 + 3.0 * m47 - 12.0 * m48;
  const double m34 = -887.0 / 5040.0 - m47 + 6.0 * m48;
  const double m35 = 3613.0 / 50400.0 + 4.0 * m47 / 5.0 - 9.0 * m48 / 5.0;
  const double m36 = 467.0 / 25200.0 - 3.0 * m47 / 5.0 + 18.0 * m48 / 5.0;
  const double m37 = 139.0 / 25200.0 - m47 / 5.0 - 9.0 * m48 / 5.0;
  const double m41 = 17.0 / 1680.0 + 2.0 * m48;
  const double m42 = -319.0 / 2520.0 + 2.0 * m47 - 8.0 * m48;
  const double m43 = -919.0 / 5040.0 - 2.0 * m47 + 6.0 * m48;
  const double m44 = -445.0 / 2016.0;
  const double m45 = 583.0 / 720.0 - m47 + 6.0 * m48;
  const double m46 = -65.0 / 224.0 - 7.0 * m48;
  const double rows[8][8] = {
      {m11, m12, m13, m14, m15, 0, 0, 0},
      {m21, m22, m23, m24, m25, m26, 0, 0},
      {m31, m32, m33, m34, m35, m36, m37, 0},
      {m41, m42, m43, m44, m45, m46, m47, m48},
      {-m48, -m47, -m46, -m45, -m44, -m43, -m42, -m41},
      {0, -m37, -m36, -m35, -m34, -m33, -m32, -m31},
      {0, 0, -m26, -m25, -m24, -m23, -m22, -m21},
      {0, 0, 0, -m15, -m14, -m13, -m12, -m11},
  };
  std::memcpy(M, rows, sizeof(rows));
}

// Sixth-order family (Section 2.2), rows/cols 1..6 <-> offsets -2..3.
void narrow6(double m36, double M[6][6]) {
  const double m11 = -11.0 / 180.0 + m36, m12 = 1.0 / 9.0 - 2.0 * m36;
  const double m13 = -1.0 / 18.0 + m36, m14 = 1.0 / 180.0;
  const double m21 = 7.0 / 60.0 - 3.0 * m36, m22 = -1.0 / 120.0 + 5.0 * m36;
  const double m23 = -17.0 / 90.0 - 2.0 * m36, m24 = 5.0 / 72.0 + m36;
  const double m25 = 1.0 / 90.0 - m36, m31 = -1.0 / 15.0 + 3.0 * m36;
  const double m32 = -11.0 / 60.0 - 3.0 * m36, m33 = -101.0 / 360.0;
  const double m34 = 137.0 / 180.0 - 2.0 * m36, m35 = -83.0 / 360.0 + m36;
  const double rows[6][6] = {
      {m11, m12, m13, m14, 0, 0},
      {m21, m22, m23, m24, m25, 0},
      {m31, m32, m33, m34, m35, m36},
      {-m36, -m35, -m34, -m33, -m32, -m31},
      {0, -m25, -m24, -m23, -m22, -m21},
      {0, 0, -m14, -m13, -m12, -m11},
  };
  std::memcpy(M, rows, sizeof(rows));
}

// d/dx (a du/dx) at the centre of nine samples: (H_{i+1/2} - H_{i-1/2})/dx^2
// with H_{i+1/2} = sum_{m,n=-3..4} a_{i+m} M_{mn} u_{i+n}   (eqs. DaDu and H).
template <class S>
S narrow(const S *a, const S *u, double dx, const double M[8][8]) {
  S hp = 0.0, hm = 0.0;
  for (int m = -3; m <= 4; ++m)
    for (int n = -3; n <= 4; ++n) {
      hp = hp + a[4 + m] * M[m + 3][n + 3] * u[4 + n];
      hm = hm + a[3 + m] * M[m + 3][n + 3] * u[3 + n];
    }
  return (hp - hm) / (dx * dx);
}

// ------------------------------------------------ physical boundaries
// Near a non-periodic boundary (Section 2.5) the stencils along its normal
// drop in order with the distance b of the cell from the boundary (b = 0 for
// the boundary cell itself):
//   b >= 4  the eighth-order stencils above;
//   b = 3   sixth-order centred first derivative and the sixth-order narrow
//           stencil (the matrix of Section 2.2 with m36 = 281/3600);
//   b = 2   fourth-order centred first derivative and the fourth-order
//           member of the narrow family (narrow4 below);
//   b = 1   advection: third-order first derivative biased away from the
//           boundary; diffusion: second-order centred (first derivative
//           (f_{i+1} - f_{i-1})/2h, second derivative with faces
//           H_{i+1/2} = (a_i + a_{i+1})(u_{i+1} - u_i)/2);
//   b = 0   advection: one-sided third-order first derivative; diffusion:
//           one-sided second-order (first derivative (-3f_0 + 4f_1 - f_2)/2h,
//           and (a u')' = a u'' + a' u' with the one-sided second-order u''
//           (2u_0 - 5u_1 + 4u_2 - u_3)/h^2 and first derivatives).
// The same formulas serve the high side mirrored (x -> -x).  Samples are
// nine values f[0..8] centred on the cell (index 4); those beyond the
// boundary are never used.
enum Kind { ADVECTION = 0, DIFFUSION = 1 };

// Fourth-order member of the narrow family: rows/cols 1..4 <-> offsets -1..2,
// exact for deg a + deg u <= 5, the corner entries zero as in the
// sixth-order matrix; one free parameter m33, set to 1/72 (it zeroes the
// a term of the h^4 truncation error; every value in [1/72, 1/24]
// minimises the sum of the absolute truncation coefficients).
void narrow4(double M[4][4]) {
  const double m33 = 1.0 / 72.0;
  const double rows[4][4] = {
      {-m33, 2.0 * m33 + 1.0 / 12.0, -m33 - 1.0 / 12.0, 0.0},
      {2.0 * m33 + 1.0 / 12.0, -3.0 * m33 - 3.0 / 4.0, 2.0 / 3.0, m33},
      {-m33, -2.0 / 3.0, 3.0 * m33 + 3.0 / 4.0, -2.0 * m33 - 1.0 / 12.0},
      {0.0, m33 + 1.0 / 12.0, -2.0 * m33 - 1.0 / 12.0, m33},
  };
  std::memcpy(M, rows, sizeof(rows));
}

// first derivative at the centre of f[0..8] for a cell at distance b from a
// boundary on side `high` (0: the boundary is below, 1: above)
template <class S>
S d1_bnd(const S *f, double dx, int b, int high, Kind kind) {
  if (b >= 4) return d1(f, dx);
  // mirror so that the boundary is below: g[o] = f[4 + o] (low) or -f[4 - o]
  S g[9];
  for (int o = -4; o <= 4; ++o) g[o + 4] = high ? S(-1.0) * f[4 - o] : f[4 + o];
  S r;
  if (b == 3)
    r = 3.0 / 4.0 * (g[5] - g[3]) - 3.0 / 20.0 * (g[6] - g[2]) + 1.0 / 60.0 * (g[7] - g[1]);
  else if (b == 2)
    r = 2.0 / 3.0 * (g[5] - g[3]) - 1.0 / 12.0 * (g[6] - g[2]);
  else if (b == 1)   // (written with differences, so a constant gives exactly 0)
    r = kind == ADVECTION ? (-2.0 * (g[3] - g[4]) + 6.0 * (g[5] - g[4]) - (g[6] - g[4])) / 6.0
                          : (g[5] - g[3]) / 2.0;
  else
    r = kind == ADVECTION ? (18.0 * (g[5] - g[4]) - 9.0 * (g[6] - g[4]) + 2.0 * (g[7] - g[4])) / 6.0
                          : (4.0 * (g[5] - g[4]) - (g[6] - g[4])) / 2.0;
  return r / dx;
}

// d/dx (a du/dx) at the centre of nine samples near a boundary
template <class S>
S narrow_bnd(const S *a, const S *u, double dx, int b, int high, const double M8[8][8]) {
  if (b >= 4) return narrow(a, u, dx, M8);
  // mirror so that the boundary is below (the operator is even in x)
  S A[9], U[9];
  for (int o = 0; o < 9; ++o) {
    A[o] = high ? a[8 - o] : a[o];
    U[o] = high ? u[8 - o] : u[o];
  }
  S hp = 0.0, hm = 0.0;
  if (b == 3) {
    double M[6][6];
    narrow6(281.0 / 3600.0, M);
    for (int m = -2; m <= 3; ++m)
      for (int n = -2; n <= 3; ++n) {
        hp = hp + A[4 + m] * M[m + 2][n + 2] * U[4 + n];
        hm = hm + A[3 + m] * M[m + 2][n + 2] * U[3 + n];
      }
  } else if (b == 2) {
    double M[4][4];
    narrow4(M);
    for (int m = -1; m <= 2; ++m)
      for (int n = -1; n <= 2; ++n) {
        hp = hp + A[4 + m] * M[m + 1][n + 1] * U[4 + n];
        hm = hm + A[3 + m] * M[m + 1][n + 1] * U[3 + n];
      }
  } else if (b == 1) {
    hp = 0.5 * (A[4] + A[5]) * (U[5] - U[4]);
    hm = 0.5 * (A[3] + A[4]) * (U[4] - U[3]);
  } else {
    // 2u_0 - 5u_1 + 4u_2 - u_3, (-3u_0 + 4u_1 - u_2)/2 and the same for a,
    // with differences from the boundary sample
    const S u2 = -5.0 * (U[5] - U[4]) + 4.0 * (U[6] - U[4]) - (U[7] - U[4]);
    const S u1 = (4.0 * (U[5] - U[4]) - (U[6] - U[4])) / 2.0;
    const S a1 = (4.0 * (A[5] - A[4]) - (A[6] - A[4])) / 2.0;
    return (A[4] * u2 + a1 * u1) / (dx * dx);
  }
  return (hp - hm) / (dx * dx);
}

// ------------------------------------------------------------ mechanism
struct Mech {
  int ns, nr;
  std::vector<double> W, nasa, A, b, Ea, Le;
  std::vector<int> nuf, nur;
  double Tlo, Thi, mu_ref, T_ref, mu_exp, Pr, bulk;
  int ref;   // -1 correction velocity, else the reference species
  int wide;  // 1: wide stencil D(a D u) for the second-derivative pairs
  int np;    // bit d: physical (non-periodic) boundaries along direction d
  double M[8][8];
  explicit Mech(const omech *m)
      : ns(m->ns), nr(m->nr), W(m->W, m->W + m->ns), nasa(m->nasa, m->nasa + 7 * m->ns),
        A(m->A, m->A + m->nr), b(m->b, m->b + m->nr), Ea(m->Ea, m->Ea + m->nr),
        Le(m->Le, m->Le + m->ns), nuf(m->nu_f, m->nu_f + m->nr * m->ns),
        nur(m->nu_r, m->nu_r + m->nr * m->ns), Tlo(m->Tlo), Thi(m->Thi), mu_ref(m->mu_ref),
        T_ref(m->T_ref), mu_exp(m->mu_exp), Pr(m->Pr), bulk(m->bulk_ratio), ref(m->ref_species),
        wide(m->wide_stencil), np(m->nonperiodic) {
    narrow8(m->m47, m->m48, M);
  }
};

// Single-range NASA-7 polynomials: c_p/R, h/(RT) (a6 = enthalpy constant),
// s/R (a7 = entropy constant).
template <class S>
S cp_R(const double *a, S T) {
  return a[0] + a[1] * T + a[2] * T * T + a[3] * T * T * T + a[4] * T * T * T * T;
}
template <class S>
S h_RT(const double *a, S T) {
  return a[0] + a[1] * T / 2.0 + a[2] * T * T / 3.0 + a[3] * T * T * T / 4.0 +
         a[4] * T * T * T * T / 5.0 + a[5] / T;
}
template <class S>
S s_R(const double *a, S T) {
  return a[0] * log(T) + a[1] * T + a[2] * T * T / 2.0 + a[3] * T * T * T / 3.0 +
         a[4] * T * T * T * T / 4.0 + a[6];
}
using std::log;
using std::exp;
using std::pow;

// Primitive and transport quantities at one cell.
template <class S>
struct Prim {
  S rho, u[3], T, p, cp;
  S mu, lam, xi;
  std::vector<S> Y, X, h, rhoD;
};

// Conserved -> primitive (Section 2.1: E is kinetic plus internal energy,
// ideal-gas mixture EOS p = rho R T sum Y_k/W_k).  Temperature from the
// internal energy by Newton's method: start at 1000 K, stop one iteration
// after the first update smaller than 1e-12 T, at most 50 iterations.
// Transport: mu = mu_ref (T/T_ref)^mu_exp, lambda = mu c_p / Pr,
// rho D_k = lambda / (c_p Le_k), bulk viscosity xi = bulk_ratio mu.
template <class S>
int prim_from_cons(const Mech &m, const S *U, Prim<S> &q) {
  const int ns = m.ns;
  q.Y.resize(ns);
  q.X.resize(ns);
  q.h.resize(ns);
  q.rhoD.resize(ns);
  q.rho = U[0];
  for (int i = 0; i < 3; ++i) q.u[i] = U[1 + i] / q.rho;
  for (int k = 0; k < ns; ++k) q.Y[k] = U[5 + k] / q.rho;
  S e = U[4] / q.rho - 0.5 * (q.u[0] * q.u[0] + q.u[1] * q.u[1] + q.u[2] * q.u[2]);
  S T = 1000.0;
  bool conv = false, done = false;
  for (int it = 0; it < 50; ++it) {
    S eT = 0.0, cv = 0.0;
    for (int k = 0; k < ns; ++k) {
      const double *a = &m.nasa[7 * k];
      const double Rk = RU / m.W[k];
      eT = eT + q.Y[k] * Rk * (T * h_RT(a, T) - T);
      cv = cv + q.Y[k] * Rk * (cp_R(a, T) - 1.0);
    }
    S dT = (eT - e) / cv;
    T = T - dT;
    if (conv) { done = true; break; }
    if (std::fabs(val(dT)) <= 1e-12 * std::fabs(val(T))) conv = true;
  }
  if (!done || !(val(T) >= m.Tlo && val(T) <= m.Thi)) return -4;
  q.T = T;
  S sumYW = 0.0;
  for (int k = 0; k < ns; ++k) sumYW = sumYW + q.Y[k] / m.W[k];
  S Wbar = 1.0 / sumYW;
  q.p = q.rho * RU * T / Wbar;
  q.cp = 0.0;
  for (int k = 0; k < ns; ++k) {
    const double *a = &m.nasa[7 * k];
    q.X[k] = q.Y[k] * Wbar / m.W[k];
    q.h[k] = RU / m.W[k] * T * h_RT(a, T);
    q.cp = q.cp + q.Y[k] * RU / m.W[k] * cp_R(a, T);
  }
  q.mu = m.mu_ref * pow(T / m.T_ref, m.mu_exp);
  q.lam = q.mu * q.cp / m.Pr;
  q.xi = m.bulk * q.mu;
  for (int k = 0; k < ns; ++k) q.rhoD[k] = q.lam / (q.cp * m.Le[k]);
  return 0;
}

// Production rates rho*omega_k (kg m^-3 s^-1): law of mass action with
// reversible Arrhenius reactions; k_f = A T^b exp(-Ea/(R T)); reverse
// constant from the equilibrium constant K_p = exp(-sum nu g/RT) and
// K_c = K_p (p_ref/(R T))^{sum nu};  q_j = k_f prod c^nu' - k_r prod c^nu'';
// rho omega_k = W_k sum_j (nu''_kj - nu'_kj) q_j, concentrations c_k = rho Y_k / W_k.
// dlnA (may be null) shifts ln A_j (used for derivatives).
template <class S>
void production(const Mech &m, S rho, S T, const S *Y, const S *dlnA, S *wdot) {
  const int ns = m.ns;
  std::vector<S> c(ns), g(ns);
  for (int k = 0; k < ns; ++k) {
    c[k] = rho * Y[k] / m.W[k];
    const double *a = &m.nasa[7 * k];
    g[k] = h_RT(a, T) - s_R(a, T);
    wdot[k] = 0.0;
  }
  for (int j = 0; j < m.nr; ++j) {
    S kf = m.A[j] * pow(T, m.b[j]) * exp(-m.Ea[j] / (RU * T));
    if (dlnA) kf = kf * exp(dlnA[j]);
    S dg = 0.0;
    int dnu = 0;
    for (int k = 0; k < ns; ++k) {
      int nu = m.nur[j * ns + k] - m.nuf[j * ns + k];
      dg = dg + double(nu) * g[k];
      dnu += nu;
    }
    S Kc = exp(-dg);
    S conc = PREF / (RU * T);
    for (int i = 0; i < dnu; ++i) Kc = Kc * conc;
    for (int i = 0; i < -dnu; ++i) Kc = Kc / conc;
    S kr = kf / Kc;
    S fwd = kf, rev = kr;
    for (int k = 0; k < ns; ++k) {
      for (int i = 0; i < m.nuf[j * ns + k]; ++i) fwd = fwd * c[k];
      for (int i = 0; i < m.nur[j * ns + k]; ++i) rev = rev * c[k];
    }
    S qj = fwd - rev;
    for (int k = 0; k < ns; ++k) {
      int nu = m.nur[j * ns + k] - m.nuf[j * ns + k];
      if (nu != 0) wdot[k] = wdot[k] + m.W[k] * double(nu) * qj;
    }
  }
}

// ------------------------------------------------------------ box state
template <class S>
struct Grid {
  int nx, ny, nz, sx, sy, sz, ns, nU;
  int np = 0;   // bit d: physical boundaries along d
  double dx[3];
  std::vector<S> U;                       // ghosted conserved state
  std::vector<S> rho, T, p, mu, lam, xi;  // primitives on the ghost grid
  std::vector<S> u[3];
  std::vector<S> Y, X, h, rhoD;           // [ns][cells]
  long n() const { return long(sx) * sy * sz; }
  long at(int i, int j, int k) const { return (long(k + NG) * sy + (j + NG)) * sx + (i + NG); }
};

int wrap(int i, int n) { return ((i % n) + n) % n; }

// Periodic ghost fill (4 layers including edges and corners) followed by the
// pointwise primitive evaluation at every stored cell.
template <class S>
int setup_grid(const Mech &m, int nx, int ny, int nz, const double *dxs, const S *Uin, Grid<S> &g) {
  g.nx = nx; g.ny = ny; g.nz = nz;
  g.sx = nx + 2 * NG; g.sy = ny + 2 * NG; g.sz = nz + 2 * NG;
  g.ns = m.ns; g.nU = 5 + m.ns;
  for (int d = 0; d < 3; ++d) g.dx[d] = dxs[d];
  const long n = g.n(), nin = long(nx) * ny * nz;
  g.np = m.np;
  // physical boundaries: at least 8 cells between them, narrow stencil only
  if (m.np && m.wide) return -1;
  const int dims[3] = {nx, ny, nz};
  for (int d = 0; d < 3; ++d)
    if (((m.np >> d) & 1) && dims[d] < 8) return -1;
  g.U.assign(long(g.nU) * n, S(0.0));
  // ghost layers: periodic images, or along a direction with physical
  // boundaries copies of the nearest boundary cell (never used by the
  // boundary stencils; they only keep the ghost primitives finite)
  auto gi = [&](int i, int nn, int d) { return (m.np >> d) & 1 ? std::min(std::max(i, 0), nn - 1) : wrap(i, nn); };
  for (int c = 0; c < g.nU; ++c)
    for (int k = -NG; k < nz + NG; ++k)
      for (int j = -NG; j < ny + NG; ++j)
        for (int i = -NG; i < nx + NG; ++i)
          g.U[c * n + g.at(i, j, k)] =
              Uin[c * nin + (long(gi(k, nz, 2)) * ny + gi(j, ny, 1)) * nx + gi(i, nx, 0)];
  g.rho.resize(n); g.T.resize(n); g.p.resize(n); g.mu.resize(n); g.lam.resize(n); g.xi.resize(n);
  for (int d = 0; d < 3; ++d) g.u[d].resize(n);
  g.Y.resize(long(m.ns) * n); g.X.resize(long(m.ns) * n);
  g.h.resize(long(m.ns) * n); g.rhoD.resize(long(m.ns) * n);
  int status = 0;
#pragma omp parallel for schedule(static) reduction(min : status)
  for (long c = 0; c < n; ++c) {
    std::vector<S> Uc(g.nU);
    for (int q = 0; q < g.nU; ++q) Uc[q] = g.U[q * n + c];
    Prim<S> pr;
    int st = prim_from_cons(m, Uc.data(), pr);
    if (st) { status = st; continue; }
    g.rho[c] = pr.rho; g.T[c] = pr.T; g.p[c] = pr.p;
    g.mu[c] = pr.mu; g.lam[c] = pr.lam; g.xi[c] = pr.xi;
    for (int d = 0; d < 3; ++d) g.u[d][c] = pr.u[d];
    for (int k = 0; k < m.ns; ++k) {
      g.Y[k * n + c] = pr.Y[k]; g.X[k * n + c] = pr.X[k];
      g.h[k * n + c] = pr.h[k]; g.rhoD[k * n + c] = pr.rhoD[k];
    }
  }
  return status;
}

// Right-hand side at one interior cell (i, j, k).
//   continuity     -sum_d D_d(rho u_d)
//   momentum i     -sum_d D_d(rho u_i u_d + p delta_id) + div tau
//   energy         -sum_d D_d((rho E + p) u_d) + div(lambda grad T) + div(tau.u) - div sum_k F_k h_k
//   species k      -sum_d D_d(rho Y_k u_d) - div F_k + rho omega_k
// Viscous stress tau_ij = eta(d_j u_i + d_i u_j - 2/3 delta_ij div u) + xi delta_ij div u
// is split into narrow second-derivative terms L_d(a, u) and mixed terms:
//   (div tau)_i = sum_d L_d(a_id, u_i) + sum_{d!=i} D_d(eta D_i u_d)
//                 + D_i((xi - 2/3 eta) sum_{j!=i} D_j u_j),
//   a_id = 4/3 eta + xi for d = i, eta otherwise;
//   div(tau.u) = sum_d [L_d(eta, |u|^2/2) + L_d(eta/3 + xi, u_d^2/2)
//                 + D_d(eta sum_{j!=d} u_j D_j u_d + (xi - 2/3 eta) u_d sum_{j!=d} D_j u_j)].
// Species flux F_k = Fbar_k - Y_k V_c with Fbar_k = -rho D_k (grad X_k + (X_k - Y_k) grad p / p)
// and V_c = sum_l Fbar_l; div Fbar_k is the narrow operator applied to the pairs
// (rho D_k, X_k) and (rho D_k (X_k-Y_k)/p, p); div(Y_k V_c) and div(h_k Y_k V_c)
// by the chain rule with div V_c = sum_l div Fbar_l.
template <class S>
void rhs_cell(const Mech &m, const Grid<S> &g, int i, int j, int k, unsigned parts, S *out) {
  const int ns = m.ns, nU = g.nU;
  const long n = g.n();
  for (int q = 0; q < nU; ++q) out[q] = 0.0;
  const long c0 = g.at(i, j, k);
  // stored index of the cell s steps along direction d (periodic images:
  // the wide operator reaches 8 cells, past the 4 ghost layers)
  // along a direction with physical boundaries: the cell's distance bd from
  // the nearer boundary and which one it is (the stencils of d1_bnd and
  // narrow_bnd); samples past the boundary are clamped copies, never used
  const int cc[3] = {i, j, k}, nn[3] = {g.nx, g.ny, g.nz};
  int bd[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    const bool phys = (g.np >> d) & 1;
    bd[d] = phys ? std::min(cc[d], nn[d] - 1 - cc[d]) : 4;
    hi[d] = phys && (nn[d] - 1 - cc[d] < cc[d]);
  }
  auto pt = [&](int d, int s) {
    int ii = i, jj = j, kk = k;
    auto mv = [&](int c, int n) { return (g.np >> d) & 1 ? std::min(std::max(c + s, 0), n - 1) : wrap(c + s, n); };
    if (d == 0) ii = mv(i, g.nx); else if (d == 1) jj = mv(j, g.ny); else kk = mv(k, g.nz);
    return g.at(ii, jj, kk);
  };
  // first derivatives along d of advective and diffusive terms
  auto dA = [&](const S *f, int d) { return d1_bnd(f, g.dx[d], bd[d], hi[d], ADVECTION); };
  auto dD = [&](const S *f, int d) { return d1_bnd(f, g.dx[d], bd[d], hi[d], DIFFUSION); };
  // D_jdir u_comp at stored index c, a cell on the line through the output
  // cell along another direction (so its position along jdir is the output
  // cell's; c has 4 neighbours or their clamped copies along jdir)
  auto grad = [&](long c, int jdir, int comp) {
    long stride = jdir == 0 ? 1 : (jdir == 1 ? g.sx : long(g.sx) * g.sy);
    S f[9];
    for (int s = -4; s <= 4; ++s) f[s + 4] = g.u[comp][c + s * stride];
    return dD(f, jdir);
  };
  // second-derivative pairs L_d(a, u): a and u sampled at s = -R..R (index
  // s + 8); narrow stencil (eq. H) from s = -4..4, or with the wide stencil
  // D(a D u): the eighth-order first derivative of a times the first
  // derivative of u, which reaches s = -8..8 (Section 2.2)
  S f[9], a[17], uu[17];
  const int R = m.wide ? 8 : 4;
  int dcur = 0;   // direction of the pairs being summed
  auto pair = [&](const S *aa, const S *uv, double h) -> S {
    if (!m.wide) return narrow_bnd(aa + 4, uv + 4, h, bd[dcur], hi[dcur], m.M);
    S g9[9];
    for (int o = -4; o <= 4; ++o) g9[o + 4] = aa[o + 8] * d1(uv + o + 4, h);
    return d1(g9, h);
  };

  if (parts & ORC_HYP) {
    for (int d = 0; d < 3; ++d) {
      for (int q = 0; q < nU; ++q) {
        for (int s = -4; s <= 4; ++s) {
          long c = pt(d, s);
          S ud = g.u[d][c];
          S fl;
          if (q == 0) fl = g.U[(1 + d) * n + c];
          else if (q <= 3) fl = g.U[q * n + c] * ud + ((q - 1) == d ? g.p[c] : S(0.0));
          else if (q == 4) fl = (g.U[4 * n + c] + g.p[c]) * ud;
          else fl = g.U[q * n + c] * ud;
          f[s + 4] = fl;
        }
        out[q] = out[q] - dA(f, d);
      }
    }
  }

  if (parts & ORC_DIFF) {
    S divVc = 0.0;
    S Vc[3];
    std::vector<S> DY(3 * ns), DhY(3 * ns);
    for (int d = 0; d < 3; ++d) {
      const double h = g.dx[d];
      dcur = d;
      // viscous momentum terms
      for (int ic = 0; ic < 3; ++ic) {
        for (int s = -R; s <= R; ++s) {
          long c = pt(d, s);
          a[s + 8] = ic == d ? 4.0 / 3.0 * g.mu[c] + g.xi[c] : g.mu[c];
          uu[s + 8] = g.u[ic][c];
        }
        out[1 + ic] = out[1 + ic] + pair(a, uu, h);
      }
      // heat conduction
      for (int s = -R; s <= R; ++s) {
        long c = pt(d, s);
        a[s + 8] = g.lam[c];
        uu[s + 8] = g.T[c];
      }
      out[4] = out[4] + pair(a, uu, h);
      // viscous work, second-derivative parts
      for (int s = -R; s <= R; ++s) {
        long c = pt(d, s);
        a[s + 8] = g.mu[c];
        uu[s + 8] = 0.5 * (g.u[0][c] * g.u[0][c] + g.u[1][c] * g.u[1][c] + g.u[2][c] * g.u[2][c]);
      }
      out[4] = out[4] + pair(a, uu, h);
      for (int s = -R; s <= R; ++s) {
        long c = pt(d, s);
        a[s + 8] = g.mu[c] / 3.0 + g.xi[c];
        uu[s + 8] = 0.5 * g.u[d][c] * g.u[d][c];
      }
      out[4] = out[4] + pair(a, uu, h);
      // mixed first-derivative parts
      for (int ic = 0; ic < 3; ++ic) {
        if (ic == d) continue;
        for (int s = -4; s <= 4; ++s) {
          long c = pt(d, s);
          f[s + 4] = g.mu[c] * grad(c, ic, d);
        }
        out[1 + ic] = out[1 + ic] + dD(f, d);
      }
      for (int s = -4; s <= 4; ++s) {
        long c = pt(d, s);
        S divt = 0.0;
        for (int jd = 0; jd < 3; ++jd)
          if (jd != d) divt = divt + grad(c, jd, jd);
        f[s + 4] = (g.xi[c] - 2.0 / 3.0 * g.mu[c]) * divt;
      }
      out[1 + d] = out[1 + d] + dD(f, d);
      for (int s = -4; s <= 4; ++s) {
        long c = pt(d, s);
        S t1 = 0.0, divt = 0.0;
        for (int jd = 0; jd < 3; ++jd) {
          if (jd == d) continue;
          t1 = t1 + g.u[jd][c] * grad(c, jd, d);
          divt = divt + grad(c, jd, jd);
        }
        f[s + 4] = g.mu[c] * t1 + (g.xi[c] - 2.0 / 3.0 * g.mu[c]) * g.u[d][c] * divt;
      }
      out[4] = out[4] + dD(f, d);
      if (m.ref >= 0) {
        // reference species (Section 2.1): species k != ref carry the mixture
        // model flux Fbar_k, the reference species carries -sum of them, and
        // the energy flux sum_k F_k h_k becomes sum_{k != ref} Fbar_k (h_k -
        // h_ref) (Section 2.4), so the pairs are (rho D_k (h_k - h_ref), X_k)
        // and (rho D_k (h_k - h_ref)(X_k - Y_k)/p, p); no correction velocity
        const int kr = m.ref;
        for (int ks = 0; ks < ns; ++ks) {
          if (ks == kr) continue;
          for (int s = -R; s <= R; ++s) {
            long c = pt(d, s);
            a[s + 8] = g.rhoD[ks * n + c];
            uu[s + 8] = g.X[ks * n + c];
          }
          S Lx = pair(a, uu, h);
          for (int s = -R; s <= R; ++s) {
            long c = pt(d, s);
            a[s + 8] = g.rhoD[ks * n + c] * (g.X[ks * n + c] - g.Y[ks * n + c]) / g.p[c];
            uu[s + 8] = g.p[c];
          }
          S Lp = pair(a, uu, h);
          out[5 + ks] = out[5 + ks] + Lx + Lp;
          out[5 + kr] = out[5 + kr] - (Lx + Lp);
          for (int s = -R; s <= R; ++s) {
            long c = pt(d, s);
            a[s + 8] = g.rhoD[ks * n + c] * (g.h[ks * n + c] - g.h[kr * n + c]);
            uu[s + 8] = g.X[ks * n + c];
          }
          out[4] = out[4] + pair(a, uu, h);
        }
        for (int s = -R; s <= R; ++s) {
          long c = pt(d, s);
          S sum = 0.0;
          for (int ks = 0; ks < ns; ++ks)
            if (ks != kr)
              sum = sum + g.rhoD[ks * n + c] * (g.h[ks * n + c] - g.h[kr * n + c]) *
                              (g.X[ks * n + c] - g.Y[ks * n + c]) / g.p[c];
          a[s + 8] = sum;
          uu[s + 8] = g.p[c];
        }
        out[4] = out[4] + pair(a, uu, h);
        continue;
      }
      // species diffusion
      for (int ks = 0; ks < ns; ++ks) {
        for (int s = -R; s <= R; ++s) {
          long c = pt(d, s);
          a[s + 8] = g.rhoD[ks * n + c];
          uu[s + 8] = g.X[ks * n + c];
        }
        S Lx = pair(a, uu, h);
        for (int s = -R; s <= R; ++s) {
          long c = pt(d, s);
          a[s + 8] = g.rhoD[ks * n + c] * (g.X[ks * n + c] - g.Y[ks * n + c]) / g.p[c];
          uu[s + 8] = g.p[c];
        }
        S Lp = pair(a, uu, h);
        out[5 + ks] = out[5 + ks] + Lx + Lp;
        divVc = divVc - (Lx + Lp);
        for (int s = -R; s <= R; ++s) {
          long c = pt(d, s);
          a[s + 8] = g.rhoD[ks * n + c] * g.h[ks * n + c];
          uu[s + 8] = g.X[ks * n + c];
        }
        out[4] = out[4] + pair(a, uu, h);
      }
      for (int s = -R; s <= R; ++s) {
        long c = pt(d, s);
        S sum = 0.0;
        for (int ks = 0; ks < ns; ++ks)
          sum = sum + g.rhoD[ks * n + c] * g.h[ks * n + c] * (g.X[ks * n + c] - g.Y[ks * n + c]) / g.p[c];
        a[s + 8] = sum;
        uu[s + 8] = g.p[c];
      }
      out[4] = out[4] + pair(a, uu, h);
      // correction velocity component d, first derivatives of Y_k and h_k Y_k
      for (int s = -4; s <= 4; ++s) f[s + 4] = g.p[pt(d, s)];
      S Dp = dD(f, d);
      S vc = 0.0;
      for (int ks = 0; ks < ns; ++ks) {
        for (int s = -4; s <= 4; ++s) f[s + 4] = g.X[ks * n + pt(d, s)];
        S DX = dD(f, d);
        vc = vc - g.rhoD[ks * n + c0] * (DX + (g.X[ks * n + c0] - g.Y[ks * n + c0]) * Dp / g.p[c0]);
        for (int s = -4; s <= 4; ++s) f[s + 4] = g.Y[ks * n + pt(d, s)];
        DY[d * ns + ks] = dD(f, d);
        for (int s = -4; s <= 4; ++s) {
          long c = pt(d, s);
          f[s + 4] = g.h[ks * n + c] * g.Y[ks * n + c];
        }
        DhY[d * ns + ks] = dD(f, d);
      }
      Vc[d] = vc;
    }
    for (int ks = 0; ks < ns && m.ref < 0; ++ks) {
      S t = g.Y[ks * n + c0] * divVc;
      for (int d = 0; d < 3; ++d) t = t + Vc[d] * DY[d * ns + ks];
      out[5 + ks] = out[5 + ks] + t;
      S te = g.h[ks * n + c0] * g.Y[ks * n + c0] * divVc;
      for (int d = 0; d < 3; ++d) te = te + Vc[d] * DhY[d * ns + ks];
      out[4] = out[4] + te;
    }
  }
}

template <class S>
void react_cell(const Mech &m, const Grid<S> &g, long c, const S *dlnA, S *out) {
  const long n = g.n();
  std::vector<S> Y(m.ns), w(m.ns);
  for (int k = 0; k < m.ns; ++k) Y[k] = g.Y[k * n + c];
  production(m, g.rho[c], g.T[c], Y.data(), dlnA, w.data());
  for (int k = 0; k < m.ns; ++k) out[5 + k] = out[5 + k] + w[k];
}

template <class S>
int rhs_all(const Mech &m, int nx, int ny, int nz, const double *dx, const S *U, unsigned parts,
            const S *dlnA, S *out, int nthreads) {
  if (nthreads > 0) omp_set_num_threads(nthreads);
  Grid<S> g;
  int st = setup_grid(m, nx, ny, nz, dx, U, g);
  if (st) return st;
  const long nin = long(nx) * ny * nz;
  const int nU = g.nU;
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j) {
      std::vector<S> o(nU);
      for (int i = 0; i < nx; ++i) {
        rhs_cell(m, g, i, j, k, parts, o.data());
        if (parts & ORC_REACT) react_cell(m, g, g.at(i, j, k), dlnA, o.data());
        long ci = (long(k) * ny + j) * nx + i;
        for (int q = 0; q < nU; ++q) out[q * nin + ci] = o[q];
      }
    }
  return 0;
}

}  // namespace

extern "C" {

void oracle_narrow_matrix(double m47, double m48, double *M) {
  double T[8][8];
  narrow8(m47, m48, T);
  std::memcpy(M, T, sizeof(T));
}

void oracle_narrow6_matrix(double m36, double *M) {
  double T[6][6];
  narrow6(m36, T);
  std::memcpy(M, T, sizeof(T));
}

double oracle_d1_point(const double *f9, double dx) { return d1(f9, dx); }

double oracle_narrow_point(const double *a9, const double *u9, double dx, double m47, double m48) {
  double M[8][8];
  narrow8(m47, m48, M);
  return narrow(a9, u9, dx, M);
}

// The boundary stencils on a line of n >= 8 points with physical boundaries
// at both ends (kind 0 advection, 1 diffusion for the first derivative).
void oracle_d1_line(int n, const double *f, double dx, int kind, double *out) {
  for (int i = 0; i < n; ++i) {
    double s[9];
    for (int o = -4; o <= 4; ++o) s[o + 4] = f[std::min(std::max(i + o, 0), n - 1)];
    const int b = std::min(i, n - 1 - i), high = (n - 1 - i) < i;
    out[i] = d1_bnd(s, dx, b, high, kind ? DIFFUSION : ADVECTION);
  }
}

void oracle_narrow_line(int n, const double *a, const double *u, double dx, double m47, double m48,
                        double *out) {
  double M[8][8];
  narrow8(m47, m48, M);
  for (int i = 0; i < n; ++i) {
    double as[9], us[9];
    for (int o = -4; o <= 4; ++o) {
      const int c = std::min(std::max(i + o, 0), n - 1);
      as[o + 4] = a[c];
      us[o + 4] = u[c];
    }
    const int b = std::min(i, n - 1 - i), high = (n - 1 - i) < i;
    out[i] = narrow_bnd(as, us, dx, b, high, M);
  }
}

void oracle_narrow4_matrix(double *M) {
  double T[4][4];
  narrow4(T);
  std::memcpy(M, T, sizeof(T));
}

void oracle_d1_periodic(int n, const double *f, double dx, double *out) {
  for (int i = 0; i < n; ++i) {
    double s[9];
    for (int o = -4; o <= 4; ++o) s[o + 4] = f[wrap(i + o, n)];
    out[i] = d1(s, dx);
  }
}

void oracle_narrow_periodic(int n, const double *a, const double *u, double dx, double m47,
                            double m48, double *out) {
  double M[8][8];
  narrow8(m47, m48, M);
  for (int i = 0; i < n; ++i) {
    double as[9], us[9];
    for (int o = -4; o <= 4; ++o) {
      as[o + 4] = a[wrap(i + o, n)];
      us[o + 4] = u[wrap(i + o, n)];
    }
    out[i] = narrow(as, us, dx, M);
  }
}

void oracle_heat2d(int n, const double *a, const double *b, const double *u, double dx,
                   double m47, double m48, double *out) {
  double M[8][8];
  narrow8(m47, m48, M);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      double as[9], bs[9], ux[9], uy[9];
      for (int o = -4; o <= 4; ++o) {
        as[o + 4] = a[j * n + wrap(i + o, n)];
        ux[o + 4] = u[j * n + wrap(i + o, n)];
        bs[o + 4] = b[wrap(j + o, n) * n + i];
        uy[o + 4] = u[wrap(j + o, n) * n + i];
      }
      out[j * n + i] = narrow(as, ux, dx, M) + narrow(bs, uy, dx, M);
    }
}

void oracle_species_thermo(const omech *om, double T, double *cp, double *h, double *s) {
  for (int k = 0; k < om->ns; ++k) {
    const double *a = om->nasa + 7 * k;
    cp[k] = cp_R(a, T);
    h[k] = h_RT(a, T);
    s[k] = s_R(a, T);
  }
}

void oracle_rate_constants(const omech *om, double T, double *kf, double *kr) {
  Mech m(om);
  for (int j = 0; j < m.nr; ++j) {
    double kfj = m.A[j] * std::pow(T, m.b[j]) * std::exp(-m.Ea[j] / (RU * T));
    double dg = 0.0;
    int dnu = 0;
    for (int k = 0; k < m.ns; ++k) {
      int nu = m.nur[j * m.ns + k] - m.nuf[j * m.ns + k];
      const double *a = &m.nasa[7 * k];
      dg += nu * (h_RT(a, T) - s_R(a, T));
      dnu += nu;
    }
    double Kc = std::exp(-dg) * std::pow(PREF / (RU * T), dnu);
    kf[j] = kfj;
    kr[j] = kfj / Kc;
  }
}

int oracle_prim_to_cons(const omech *om, long ncell, const double *p, const double *T,
                        const double *Y, const double *u, double *U) {
  Mech m(om);
  const int ns = m.ns;
  for (long c = 0; c < ncell; ++c) {
    double sumYW = 0.0;
    for (int k = 0; k < ns; ++k) sumYW += Y[k * ncell + c] / m.W[k];
    double Wbar = 1.0 / sumYW;
    double rho = p[c] * Wbar / (RU * T[c]);
    double e = 0.0;
    for (int k = 0; k < ns; ++k) {
      const double *a = &m.nasa[7 * k];
      e += Y[k * ncell + c] * RU / m.W[k] * (T[c] * h_RT(a, T[c]) - T[c]);
    }
    double ke = 0.5 * (u[c] * u[c] + u[ncell + c] * u[ncell + c] + u[2 * ncell + c] * u[2 * ncell + c]);
    U[c] = rho;
    for (int i = 0; i < 3; ++i) U[(1 + i) * ncell + c] = rho * u[i * ncell + c];
    U[4 * ncell + c] = rho * (e + ke);
    for (int k = 0; k < ns; ++k) U[(5 + k) * ncell + c] = rho * Y[k * ncell + c];
  }
  return 0;
}

int oracle_cons_to_prim(const omech *om, long ncell, const double *U, double *out) {
  Mech m(om);
  const int nU = 5 + m.ns;
  int status = 0;
  std::vector<double> Uc(nU);
  for (long c = 0; c < ncell; ++c) {
    for (int q = 0; q < nU; ++q) Uc[q] = U[q * ncell + c];
    Prim<double> pr;
    int st = prim_from_cons(m, Uc.data(), pr);
    if (st) { status = st; continue; }
    out[c] = pr.rho;
    for (int i = 0; i < 3; ++i) out[(1 + i) * ncell + c] = pr.u[i];
    out[4 * ncell + c] = pr.T;
    out[5 * ncell + c] = pr.p;
  }
  return status;
}

int oracle_sound_speed(const omech *om, long ncell, const double *U, double *c_out) {
  Mech m(om);
  const int nU = 5 + m.ns;
  int status = 0;
#pragma omp parallel for schedule(static) reduction(min : status)
  for (long c = 0; c < ncell; ++c) {
    std::vector<double> Uc(nU);
    for (int q = 0; q < nU; ++q) Uc[q] = U[q * ncell + c];
    Prim<double> pr;
    int st = prim_from_cons(m, Uc.data(), pr);
    if (st) { status = st; continue; }
    double Rmix = pr.p / (pr.rho * pr.T);
    double gamma = pr.cp / (pr.cp - Rmix);
    c_out[c] = std::sqrt(gamma * pr.p / pr.rho);
  }
  return status;
}

int oracle_production(const omech *om, long ncell, const double *U, double *wdot) {
  Mech m(om);
  const int nU = 5 + m.ns;
  int status = 0;
  std::vector<double> Uc(nU), w(m.ns);
  for (long c = 0; c < ncell; ++c) {
    for (int q = 0; q < nU; ++q) Uc[q] = U[q * ncell + c];
    Prim<double> pr;
    int st = prim_from_cons(m, Uc.data(), pr);
    if (st) { status = st; continue; }
    production(m, pr.rho, pr.T, pr.Y.data(), (const double *)nullptr, w.data());
    for (int k = 0; k < m.ns; ++k) wdot[k * ncell + c] = w[k];
  }
  return status;
}

int oracle_rhs(const omech *om, int nx, int ny, int nz, double dx, double dy, double dz,
               const double *U, unsigned parts, double *out, int nthreads) {
  if (nx < 1 || ny < 1 || nz < 1) return -1;
  Mech m(om);
  const double h[3] = {dx, dy, dz};
  return rhs_all<double>(m, nx, ny, nz, h, U, parts, nullptr, out, nthreads);
}

int oracle_rhs_cells(const omech *om, int nx, int ny, int nz, double dx, double dy, double dz,
                     const double *U, unsigned parts, int ncells, const int *cells, double *out,
                     int nthreads) {
  if (nx < 1 || ny < 1 || nz < 1) return -1;
  if (nthreads > 0) omp_set_num_threads(nthreads);
  Mech m(om);
  const double h[3] = {dx, dy, dz};
  Grid<double> g;
  int st = setup_grid(m, nx, ny, nz, h, U, g);
  if (st) return st;
  const int nU = g.nU;
#pragma omp parallel for schedule(dynamic)
  for (int c = 0; c < ncells; ++c) {
    int i = cells[3 * c], j = cells[3 * c + 1], k = cells[3 * c + 2];
    std::vector<double> o(nU);
    rhs_cell(m, g, i, j, k, parts, o.data());
    if (parts & ORC_REACT) react_cell(m, g, g.at(i, j, k), (const double *)nullptr, o.data());
    for (int q = 0; q < nU; ++q) out[long(c) * nU + q] = o[q];
  }
  return 0;
}

int oracle_rhs_jvp(const omech *om, int nx, int ny, int nz, double dx, double dy, double dz,
                   const double *U, const double *wU, const double *wA, unsigned parts,
                   double *out, double *jvp, int nthreads) {
  if (nx < 1 || ny < 1 || nz < 1) return -1;
  Mech m(om);
  const double h[3] = {dx, dy, dz};
  const long nin = long(nx) * ny * nz;
  const int nU = 5 + m.ns;
  std::vector<dual> Ud(nU * nin), od(nU * nin), dA(m.nr);
  for (long c = 0; c < nU * nin; ++c) Ud[c] = dual(U[c], wU ? wU[c] : 0.0);
  for (int j = 0; j < m.nr; ++j) dA[j] = dual(0.0, wA ? wA[j] : 0.0);
  int st = rhs_all<dual>(m, nx, ny, nz, h, Ud.data(), parts, dA.data(), od.data(), nthreads);
  if (st) return st;
  for (long c = 0; c < nU * nin; ++c) {
    if (out) out[c] = od[c].v;
    jvp[c] = od[c].d;
  }
  return 0;
}

int oracle_rhs_jvp_cells(const omech *om, int nx, int ny, int nz, double dx, double dy, double dz,
                         const double *U, const double *wU, const double *wA, unsigned parts,
                         int ncells, const int *cells, double *jvp, int nthreads) {
  if (nx < 1 || ny < 1 || nz < 1) return -1;
  if (nthreads > 0) omp_set_num_threads(nthreads);
  Mech m(om);
  const double h[3] = {dx, dy, dz};
  const long nin = long(nx) * ny * nz;
  const int nU = 5 + m.ns;
  std::vector<dual> Ud(nU * nin), dA(m.nr);
  for (long c = 0; c < nU * nin; ++c) Ud[c] = dual(U[c], wU ? wU[c] : 0.0);
  for (int j = 0; j < m.nr; ++j) dA[j] = dual(0.0, wA ? wA[j] : 0.0);
  Grid<dual> g;
  int st = setup_grid(m, nx, ny, nz, h, Ud.data(), g);
  if (st) return st;
#pragma omp parallel for schedule(dynamic)
  for (int c = 0; c < ncells; ++c) {
    int i = cells[3 * c], j = cells[3 * c + 1], k = cells[3 * c + 2];
    std::vector<dual> o(nU);
    rhs_cell(m, g, i, j, k, parts, o.data());
    if (parts & ORC_REACT) react_cell(m, g, g.at(i, j, k), dA.data(), o.data());
    for (int q = 0; q < nU; ++q) jvp[long(c) * nU + q] = o[q].d;
  }
  return 0;
}

}  // extern "C"
