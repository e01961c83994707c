// Device building blocks shared by the forward and adjoint kernels:
// layout of the primitive fields, eighth-order first derivative, NASA-7
// thermodynamics, the Newton temperature solve, the chemistry source and the
// narrow-stencil face-difference matrix.
#pragma once
#include <math.h>

#include "nsdc_internal.h"

namespace nsdc {

// e^x for the reaction rates: x = k ln2/64 + r with k = rint(64 x / ln 2) and
// |r| <= ln2/128 (Cody-Waite reduction with a two-part ln2/64 whose leading
// part has 37 significant bits, so k times it is exact for |k| < 2^16), e^r
// by its Taylor polynomial to degree 5 (truncation below 4e-17 relative),
// 2^(j/64), j = k mod 64, from the table tab (correctly rounded entries) and
// 2^floor(k/64) by ldexp (which also gives the overflow and underflow
// limits).  Error within about one ulp.
constexpr double EXP_INV_LN2_64 = 92.33248261689366;        // 64 / ln 2
constexpr double EXP_LN2_64_HI = 0.010830424696223417;      // 0x3f862e42fefa0000
constexpr double EXP_LN2_64_LO = 2.572804622327669e-14;     // ln2/64 - HI
__host__ __device__ __forceinline__ double exp_tab(double x, const double *tab) {
  const double kd = rint(x * EXP_INV_LN2_64);
  const int k = (int)kd;
  double r = fma(-kd, EXP_LN2_64_HI, x);
  r = fma(-kd, EXP_LN2_64_LO, r);
  // e^r - 1 = r (1 + r/2 + r^2/6 + r^3/24 + r^4/120), added to the table
  // entry t as t + t (e^r - 1) so only the last rounding falls on the result
  double p = fma(r, 1.0 / 120.0, 1.0 / 24.0);
  p = fma(r, p, 1.0 / 6.0);
  p = fma(r, p, 0.5);
  p = fma(r, p, 1.0);
  const double t = tab[k & 63];
  return ldexp(fma(t, r * p, t), k >> 6);
}
// eighth-order centred first-derivative weights
constexpr double C1 = 4.0 / 5.0, C2 = -1.0 / 5.0, C3 = 4.0 / 105.0, C4 = -1.0 / 280.0;

template <int NS>
struct Layout {
  static constexpr int NU = 5 + NS;
  // primitive fields stored per cell
  static constexpr int PU = 0, PV = 1, PW = 2, PT = 3, PP = 4, PMU = 5, PLAM = 6, PRD = 7;
  static constexpr int PY = 8, PX = 8 + NS, PH = 8 + 2 * NS, PWB = 8 + 3 * NS;
  static constexpr int NP = prim_fields(NS);
  static_assert(NP == PWB + 1, "the primitive field count follows the layout");
};

__device__ __forceinline__ double d1(const double *f, double idx) {
  return (C1 * (f[5] - f[3]) + C2 * (f[6] - f[2]) + C3 * (f[7] - f[1]) + C4 * (f[8] - f[0])) * idx;
}

// ---------------------------------------------------------- thermodynamics
__device__ __forceinline__ double cp_R(const DevMech *__restrict__ m, int k, double T) {
  const double *a = m->cp[k];
  return a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
}
__device__ __forceinline__ double h_RT(const DevMech *__restrict__ m, int k, double T, double invT) {
  const double *a = m->hc[k];
  return a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4]))) + m->h6[k] * invT;
}
// g/(RT) of the reaction-rate equilibrium constants from the combined
// coefficients (the h/(RT) and s/R polynomials folded into one)
__device__ __forceinline__ double g_RT(const DevMech *__restrict__ m, int k, double T, double invT, double lnT) {
  const double *c = m->gc[k];
  return fma(m->h6[k], invT, fma(-m->cp[k][0], lnT, fma(T, c[1] + T * (c[2] + T * (c[3] + T * c[4])), c[0])));
}
__device__ __forceinline__ double s_R(const DevMech *__restrict__ m, int k, double T, double lnT) {
  const double *a = m->sc[k];
  return m->cp[k][0] * lnT + T * (a[0] + T * (a[1] + T * (a[2] + T * a[3]))) + m->s7[k];
}

// Temperature from the specific internal energy e by Newton's method on
// e(T) = sum_k Y_k R_k T (h_k/(R_k T) - 1), de/dT = c_v: start at T0 (1000 K
// unless a nearby temperature is known), stop one iteration after the first
// update below 1e-12 T (at most 50).  With one NASA-7 range per species e(T)
// is a quintic in T whose coefficients are the mass-weighted species
// coefficients, so the mixture is summed once and every iteration evaluates
// two short polynomials (e and its derivative, which is c_v).
// e(T) = c5 + T (c0 + T (c1 + T (c2 + T (c3 + T c4)))): the mixture's
// coefficients, sum_k Y_k R_k times the species' (a1 - 1, a2/2, a3/3, a4/4,
// a5/5, a6), over the species k = K0, K0 + KS, ... in increasing order.
template <int NS, int K0 = 0, int KS = 1>
__device__ __forceinline__ void e_coeffs(const DevMech *__restrict__ m, const double *Y, double *c) {
  // keep the coefficient loads here: hoisted into an enclosing loop, the
  // mechanism tables exceed the scalar registers and are spilled
  asm volatile("" ::: "memory");
#pragma unroll
  for (int i = 0; i < 6; ++i) c[i] = 0.0;
#pragma unroll
  for (int k = K0; k < NS; k += KS) {
    const double YR = Y[k] * m->Rk[k];
    const double *a = m->hc[k];
    c[0] += YR * (a[0] - 1.0);
    c[1] += YR * a[1];
    c[2] += YR * a[2];
    c[3] += YR * a[3];
    c[4] += YR * a[4];
    c[5] += YR * m->h6[k];
  }
}
// Newton's method on e(T) = e from the mixture's coefficients c, de/dT = c_v:
// start at T0, stop one iteration after the first update below 1e-12 T (at
// most 50).
__device__ __forceinline__ int temperature_c(const DevMech *__restrict__ m, const double *c, double e, double &T,
                                             double T0) {
  const double c0 = c[0], c1 = c[1], c2 = c[2], c3 = c[3], c4 = c[4], c5 = c[5];
  const double d1 = 2.0 * c1, d2 = 3.0 * c2, d3 = 4.0 * c3, d4 = 5.0 * c4;
  T = T0;
  bool conv = false;
  for (int it = 0; it < 50; ++it) {
    const double eT = c5 + T * (c0 + T * (c1 + T * (c2 + T * (c3 + T * c4))));
    const double cv = c0 + T * (d1 + T * (d2 + T * (d3 + T * d4)));
    const double dT = (eT - e) / cv;
    T -= dT;
    if (conv) return (T >= m->Tlo && T <= m->Thi) ? 0 : NSDC_ERR_TRANGE;
    if (fabs(dT) <= 1e-12 * fabs(T)) conv = true;
  }
  return NSDC_ERR_NEWTON;
}
template <int NS>
__device__ int temperature(const DevMech *__restrict__ m, const double *Y, double e, double &T,
                           double T0 = 1000.0) {
  double c[6];
  e_coeffs<NS>(m, Y, c);
  return temperature_c(m, c, e, T, T0);
}

// Chemistry source rho omega_k (mass action, reversible Arrhenius reactions,
// reverse rate from the equilibrium constant of the Gibbs energies):
//   k_r = k_f exp(sum nu g/RT) (R T / p_ref)^{sum nu}.
// Every reaction has two reactant and two product slots; an absent molecule
// points at slot NS, a dummy species.  The rate of progress is formed with
// one exponential per reaction: with G_k = g_k/RT, b_k = c_k exp(G_k) and the
// dummy slot's G = -ln(R T / p_ref), c = 1 (so that sum nu, the absent
// reactant molecules minus the absent product molecules, is carried by the
// slots),
//   q = k_f c_r0 c_r1 - k_r c_p0 c_p1 = exp(ln k_f - G_r0 - G_r1) (b_r0 b_r1 - b_p0 b_p1),
// and the exponent is one polynomial in T per reaction (DevMech::xc, the
// reactants' NASA coefficients folded in).  Per cell that costs NS + 1
// exponentials for the b_k instead of one more per reaction.
__device__ __forceinline__ double rate_exponent(const DevMech *__restrict__ m, int j, double T, double invT,
                                                double lnT) {
  const double *x = m->xc[j];
  return fma(x[2], invT, fma(x[1], lnT, fma(T, x[3] + T * (x[4] + T * (x[5] + T * x[6])), x[0])));
}
template <int NS>
__device__ void production(const DevMech *__restrict__ m, double rho, double T, const double *Y,
                           double *wdot) {
  double b[NS + 1], w[NS + 1];
  const double lnT = log(T), invT = 1.0 / T;
  const double lnRTp = lnT + LN_RU_PREF;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    b[k] = rho * Y[k] * m->invW[k] * exp(g_RT(m, k, T, invT, lnT));
    w[k] = 0.0;
  }
  b[NS] = exp(-lnRTp);
  w[NS] = 0.0;
  const int nr = m->nr;
#pragma unroll 2
  for (int j = 0; j < nr; ++j) {
    const int r0 = m->rs[j][0], r1 = m->rs[j][1], p0 = m->ps[j][0], p1 = m->ps[j][1];
    const double q = exp(rate_exponent(m, j, T, invT, lnT)) * (b[r0] * b[r1] - b[p0] * b[p1]);
    w[r0] -= q;
    w[r1] -= q;
    w[p0] += q;
    w[p1] += q;
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) wdot[k] = w[k] * m->W[k];
}

// The same source with the per-cell arrays b, G and w in this thread's LDS
// column: entry k of array a at sh[(a (NS+1) + k) 256] (consecutive threads
// own consecutive doubles).  A species index then costs one address add
// shared by the three arrays, instead of indexed register moves.  Here the
// exponent is ln k_f - G_r0 - G_r1 from the cell's G_k (two LDS reads instead
// of production()'s seven-coefficient polynomial per reaction: the faster
// form with a lane per cell).  The exponentials use exp_tab with the
// workgroup's copy of the 2^(j/64) table (64 doubles after the three arrays).
template <int NS, int LIMIT = 65536>
constexpr bool chem_in_lds() {
  return (3 * (NS + 1) * 256 + 64) * sizeof(double) <= LIMIT;
}
template <int NS>
__device__ void production_sh(const DevMech *__restrict__ m, double rho, double T, const double *Y,
                              double *wdot, double *sh, const double *tab) {
  constexpr int S = 256, A = (NS + 1) * S;
  const double lnT = log(T), invT = 1.0 / T;
  const double lnRTp = lnT + LN_RU_PREF;
  asm volatile("" ::: "memory");
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double g = g_RT(m, k, T, invT, lnT);
    sh[A + k * S] = g;
    sh[k * S] = rho * Y[k] * m->invW[k] * exp_tab(g, tab);
    sh[2 * A + k * S] = 0.0;
  }
  sh[A + NS * S] = -lnRTp;
  sh[NS * S] = exp_tab(-lnRTp, tab);
  sh[2 * A + NS * S] = 0.0;
  const int nr = m->nr;
#pragma unroll 4
  for (int j = 0; j < nr; ++j) {
    const int r0 = m->rs[j][0] * S, r1 = m->rs[j][1] * S, p0 = m->ps[j][0] * S, p1 = m->ps[j][1] * S;
    const double lnkf = m->lnA[j] + m->beta[j] * lnT - m->EaR[j] * invT;
    const double kf = exp_tab(lnkf - (sh[A + r0] + sh[A + r1]), tab);
    const double q = kf * (sh[r0] * sh[r1] - sh[p0] * sh[p1]);
    atomicAdd(sh + 2 * A + r0, -q);
    atomicAdd(sh + 2 * A + r1, -q);
    atomicAdd(sh + 2 * A + p0, q);
    atomicAdd(sh + 2 * A + p1, q);
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) wdot[k] = sh[2 * A + k * S] * m->W[k];
}

// Chemistry source through the LDS column when the block's arrays fit in
// LIMIT bytes (sh: this thread's column of a [3][NS+1][256] shared array
// followed by the 2^(j/64) table, from chem_lds_setup), else in registers.
template <int NS, int LIMIT = 65536>
__device__ __forceinline__ void production_any(const DevMech *__restrict__ m, double rho, double T,
                                               const double *Y, double *wdot, double *sh) {
  if constexpr (chem_in_lds<NS, LIMIT>())
    production_sh<NS>(m, rho, T, Y, wdot, sh, sh - threadIdx.x + 3 * (NS + 1) * 256);
  else
    production<NS>(m, rho, T, Y, wdot);
}
#define NSDC_CHEM_LDS(NS, LIMIT, name) \
  __shared__ double name[chem_in_lds<NS, LIMIT>() ? 3 * ((NS) + 1) * 256 + 64 : 1]
// This thread's chemistry column in the LDS array `base` (NSDC_CHEM_LDS),
// once the workgroup has copied the 2^(j/64) table behind the three arrays.
// Every thread of the workgroup must call it, before any work-item loop.
template <int NS, int LIMIT>
__device__ __forceinline__ double *chem_lds_setup(double *base, const DevMech *__restrict__ m) {
  if constexpr (chem_in_lds<NS, LIMIT>()) {
    double *tab = base + 3 * (NS + 1) * 256;
    for (int j = threadIdx.x; j < 64; j += blockDim.x) tab[j] = m->e2tab[j];
    __syncthreads();
    return base + threadIdx.x;
  } else {
    return base;
  }
}

// Conserved state of one cell -> density, velocity, mass fractions and
// temperature.  Returns an error bit mask (0 = ok).
template <int NS>
__device__ int cell_state(const DevMech *__restrict__ m, const double *Uc, double &rho, double *u,
                          double *Y, double &T, double T0 = 1000.0) {
  rho = Uc[0];
  const double ir = 1.0 / rho;
  u[0] = Uc[1] * ir;
  u[1] = Uc[2] * ir;
  u[2] = Uc[3] * ir;
#pragma unroll
  for (int k = 0; k < NS; ++k) Y[k] = Uc[5 + k] * ir;
  const double e = Uc[4] * ir - 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  int err = rho > 0.0 ? 0 : NSDC_ERR_RHO;
  err |= temperature<NS>(m, Y, e, T, T0);
  return err;
}

// cell_state with the mixture's energy coefficients summed as the lane pairs
// of the fine sweep sum them: over the even and the odd species apart, then
// the two partial sums added.
template <int NS>
__device__ int cell_state_pair(const DevMech *__restrict__ m, const double *Uc, double &rho, double *u,
                               double *Y, double &T, double T0) {
  rho = Uc[0];
  const double ir = 1.0 / rho;
  u[0] = Uc[1] * ir;
  u[1] = Uc[2] * ir;
  u[2] = Uc[3] * ir;
#pragma unroll
  for (int k = 0; k < NS; ++k) Y[k] = Uc[5 + k] * ir;
  const double e = Uc[4] * ir - 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  double c0[6], c1[6], c[6];
  e_coeffs<NS, 0, 2>(m, Y, c0);
  e_coeffs<NS, 1, 2>(m, Y, c1);
#pragma unroll
  for (int q = 0; q < 6; ++q) c[q] = c0[q] + c1[q];
  int err = rho > 0.0 ? 0 : NSDC_ERR_RHO;
  err |= temperature_c(m, c, e, T, T0);
  return err;
}

__device__ __forceinline__ bool tile_cell(const Item &w, TileShape ts, int &x, int &y, int &z) {
  const int t = threadIdx.x;
  x = w.x0 + t % ts.tx;
  y = w.y0 + (t / ts.tx) % ts.ty;
  z = w.z0 + t / (ts.tx * ts.ty);
  return true;
}

// The narrow operator at the centre of nine samples, written through the 9x9
// face-difference matrix B: (H_{i+1/2} - H_{i-1/2}) = sum_{o,c} a_o B_oc u_c with
// B_oc = M_{o-1,c-1} - M_{o,c} (eqs. DaDu, H).  bvec computes v = B u once per
// field (B is banded: row o spans columns o-4..o+4); every coefficient paired
// with that field then costs a nine-term dot product.
//
// For the paper's default free parameters (m47 = 3557/44100, m48 =
// -2083/117600) B is a compile-time table, so its entries are instruction
// constants; other parameter values read B from the mechanism tables.
struct Mat9 {
  double v[9][9];
};
constexpr Mat9 smc_face_matrix() {
  const double a47 = 3557.0 / 44100.0, a48 = -2083.0 / 117600.0;
  const double top[4][8] = {
      {5.0 / 336 + a48, -83.0 / 3600 - a47 / 5 - 14 * a48 / 5, 299.0 / 50400 + 2 * a47 / 5 + 13 * a48 / 5,
       17.0 / 12600 - a47 / 5 - 4 * a48 / 5, 1.0 / 1120, 0, 0, 0},
      {-11.0 / 560 - 2 * a48, -31.0 / 360 + a47 + 3 * a48, 41.0 / 200 - 9 * a47 / 5 + 4 * a48 / 5,
       -5927.0 / 50400 + 4 * a47 / 5 - 9 * a48 / 5, 17.0 / 600 - a47 / 5 - 4 * a48 / 5,
       -503.0 / 50400 + a47 / 5 + 4 * a48 / 5, 0, 0},
      {-1.0 / 280, 1097.0 / 5040 - 2 * a47 + 6 * a48, -1349.0 / 10080 + 3 * a47 - 12 * a48,
       -887.0 / 5040 - a47 + 6 * a48, 3613.0 / 50400 + 4 * a47 / 5 - 9 * a48 / 5,
       467.0 / 25200 - 3 * a47 / 5 + 18 * a48 / 5, 139.0 / 25200 - a47 / 5 - 9 * a48 / 5, 0},
      {17.0 / 1680 + 2 * a48, -319.0 / 2520 + 2 * a47 - 8 * a48, -919.0 / 5040 - 2 * a47 + 6 * a48,
       -445.0 / 2016, 583.0 / 720 - a47 + 6 * a48, -65.0 / 224 - 7 * a48, a47, a48},
  };
  double M[8][8] = {};
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 8; ++c) {
      M[r][c] = top[r][c];
      M[7 - r][7 - c] = -top[r][c];
    }
  Mat9 B = {};
  for (int o = 0; o < 9; ++o)
    for (int c = 0; c < 9; ++c)
      B.v[o][c] = ((o >= 1 && c >= 1) ? M[o - 1][c - 1] : 0.0) - ((o <= 7 && c <= 7) ? M[o][c] : 0.0);
  return B;
}
constexpr Mat9 SMC_B = smc_face_matrix();

template <bool FIXED>
__device__ __forceinline__ void bvec(const DevMech *__restrict__ m, const double *u, double *v) {
#pragma unroll
  for (int o = 0; o < 9; ++o) {
    double acc = 0.0;
#pragma unroll
    for (int c = (o > 4 ? o - 4 : 0); c <= (o < 4 ? o + 4 : 8); ++c)
      acc += (FIXED ? SMC_B.v[o][c] : m->B[o][c]) * u[c];
    v[o] = acc;
  }
}
__device__ __forceinline__ double dot9(const double *a, const double *v) {
  double s = 0.0;
#pragma unroll
  for (int o = 0; o < 9; ++o) s += a[o] * v[o];
  return s;
}
// first derivative of the pointwise product a*b
__device__ __forceinline__ double d1p(const double *a, const double *b, double idx) {
  return (C1 * (a[5] * b[5] - a[3] * b[3]) + C2 * (a[6] * b[6] - a[2] * b[2]) +
          C3 * (a[7] * b[7] - a[1] * b[1]) + C4 * (a[8] * b[8] - a[0] * b[0])) * idx;
}

}  // namespace nsdc
