// Device kernels of the reacting Navier-Stokes right-hand side and of the
// (multirate) spectral deferred correction step, FP64, gfx950.
//
// Every kernel walks a list of work items (box, tile origin) with a
// grid-stride loop, so one launch covers one box or a whole batch of boxes
// of different sizes.  Fields are component-major with x fastest; state and
// primitive arrays carry 4 ghost layers ("stored" cells), right-hand sides
// and SDC node values are interior-only.
//
// Stages of one right-hand-side evaluation (Section 2 of the paper):
//   k_ghost    periodic fill of the 4 ghost layers (edges and corners too)
//   k_prims    conserved -> primitive variables at every stored cell:
//              Newton solve of e(T) = sum_k Y_k e_k(T), ideal-gas EOS, mole
//              fractions, species enthalpies, transport coefficients; on the
//              interior it also initialises dU/dt (zero or the chemistry
//              source rho omega_k)
//   k_vgrad    eighth-order velocity gradient D_j u_i where a later stage
//              needs it (at the ghost points along the other directions)
//   k_dir<D>   every term that differentiates along direction D: convective
//              flux divergence, the narrow second-derivative operator for
//              all (coefficient, field) pairs, the mixed viscous terms, and
//              the direction-D share of the correction-velocity terms
//              (which separate by direction: Y_k div V_c + V_c . grad Y_k is
//              a sum over D of Y_k (div V_c)_D + V_c,D D_D Y_k).
#include <math.h>

#include "nsdc_internal.h"

namespace nsdc {

constexpr double RU = 8.31446261815324;
constexpr double PREF = 101325.0;
// eighth-order centred first-derivative weights
constexpr double C1 = 4.0 / 5.0, C2 = -1.0 / 5.0, C3 = 4.0 / 105.0, C4 = -1.0 / 280.0;

template <int NS>
struct Layout {
  static constexpr int NU = 5 + NS;
  // primitive fields stored per cell
  static constexpr int PU = 0, PV = 1, PW = 2, PT = 3, PP = 4, PMU = 5, PLAM = 6, PRD = 7;
  static constexpr int PY = 8, PX = 8 + NS, PH = 8 + 2 * NS;
  static constexpr int NP = 8 + 3 * NS;
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
__device__ __forceinline__ double s_R(const DevMech *__restrict__ m, int k, double T, double lnT) {
  const double *a = m->sc[k];
  return m->cp[k][0] * lnT + T * (a[0] + T * (a[1] + T * (a[2] + T * a[3]))) + m->s7[k];
}

// Temperature from the specific internal energy e by Newton's method on
// e(T) = sum_k Y_k R_k T (h_k/(R_k T) - 1), dE/dT = c_v: start at 1000 K,
// stop one iteration after the first update below 1e-12 T (at most 50).
template <int NS>
__device__ int temperature(const DevMech *__restrict__ m, const double *Y, double e, double &T) {
  T = 1000.0;
  bool conv = false;
  for (int it = 0; it < 50; ++it) {
    const double invT = 1.0 / T;
    double eT = 0.0, cv = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const double YR = Y[k] * m->Rk[k];
      eT += YR * T * (h_RT(m, k, T, invT) - 1.0);
      cv += YR * (cp_R(m, k, T) - 1.0);
    }
    const double dT = (eT - e) / cv;
    T -= dT;
    if (conv) return (T >= m->Tlo && T <= m->Thi) ? 0 : NSDC_ERR_TRANGE;
    if (fabs(dT) <= 1e-12 * fabs(T)) conv = true;
  }
  return NSDC_ERR_NEWTON;
}

// Chemistry source rho omega_k (mass action, reversible Arrhenius reactions,
// reverse rate from the equilibrium constant of the Gibbs energies):
//   k_r = k_f exp(sum nu g/RT) (R T / p_ref)^{sum nu}.
template <int NS>
__device__ void production(const DevMech *__restrict__ m, double rho, double T, const double *Y,
                           double *wdot) {
  double c[NS], g[NS], w[NS];
  const double lnT = log(T), invT = 1.0 / T;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    c[k] = rho * Y[k] * m->invW[k];
    g[k] = h_RT(m, k, T, invT) - s_R(m, k, T, lnT);
    w[k] = 0.0;
  }
  const double lnRTp = log(RU * T / PREF);
  const int nr = m->nr;
  for (int j = 0; j < nr; ++j) {
    const int r0 = m->rs[j][0], r1 = m->rs[j][1], p0 = m->ps[j][0], p1 = m->ps[j][1];
    const double lnkf = m->lnA[j] + m->beta[j] * lnT - m->EaR[j] * invT;
    double dg = g[p0] - g[r0];
    if (p1 >= 0) dg += g[p1];
    if (r1 >= 0) dg -= g[r1];
    const double kf = exp(lnkf);
    const double kr = exp(lnkf + dg + m->dnu[j] * lnRTp);
    double fwd = kf * c[r0];
    if (r1 >= 0) fwd *= c[r1];
    double rev = kr * c[p0];
    if (p1 >= 0) rev *= c[p1];
    const double q = fwd - rev;
    w[r0] -= q;
    if (r1 >= 0) w[r1] -= q;
    w[p0] += q;
    if (p1 >= 0) w[p1] += q;
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) wdot[k] = w[k] * m->W[k];
}

// Conserved state of one cell -> density, velocity, mass fractions and
// temperature.  Returns an error bit mask (0 = ok).
template <int NS>
__device__ int cell_state(const DevMech *__restrict__ m, const double *Uc, double &rho, double *u,
                          double *Y, double &T) {
  rho = Uc[0];
  const double ir = 1.0 / rho;
  u[0] = Uc[1] * ir;
  u[1] = Uc[2] * ir;
  u[2] = Uc[3] * ir;
#pragma unroll
  for (int k = 0; k < NS; ++k) Y[k] = Uc[5 + k] * ir;
  const double e = Uc[4] * ir - 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  int err = rho > 0.0 ? 0 : NSDC_ERR_RHO;
  err |= temperature<NS>(m, Y, e, T);
  return err;
}

__device__ __forceinline__ bool tile_cell(const Item &w, TileShape ts, int &x, int &y, int &z) {
  const int t = threadIdx.x;
  x = w.x0 + t % ts.tx;
  y = w.y0 + (t / ts.tx) % ts.ty;
  z = w.z0 + t / (ts.tx * ts.ty);
  return true;
}

// ------------------------------------------------------------------ kernels
template <int NS>
__global__ __launch_bounds__(256) void k_prim_to_cons(const BoxDev *__restrict__ boxes,
                                                      const Item *__restrict__ items, int nitems,
                                                      TileShape ts, const double *__restrict__ p,
                                                      const double *__restrict__ T,
                                                      const double *__restrict__ Y,
                                                      const double *__restrict__ u, FRef Uref,
                                                      const DevMech *__restrict__ m) {
  constexpr int NU = 5 + NS;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int x, y, z;
    tile_cell(w, ts, x, y, z);
    if (x >= b.nx || y >= b.ny || z >= b.nz) continue;
    const long long nI = (long long)b.nx * b.ny * b.nz, nS = (long long)b.sx * b.sy * b.sz;
    const long long i = ((long long)z * b.ny + y) * b.nx + x;
    const long long s = ((long long)(z + NSDC_NG) * b.sy + (y + NSDC_NG)) * b.sx + (x + NSDC_NG);
    double *U = Uref.get(w.box, b.offS * NU);
    const double Tc = T[i], invT = 1.0 / Tc;
    double Yk[NS], sumYW = 0.0, e = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      Yk[k] = Y[k * nI + i];
      sumYW += Yk[k] * m->invW[k];
      e += Yk[k] * m->Rk[k] * Tc * (h_RT(m, k, Tc, invT) - 1.0);
    }
    const double rho = p[i] / (RU * Tc * sumYW);
    const double ux = u[i], uy = u[nI + i], uz = u[2 * nI + i];
    U[s] = rho;
    U[nS + s] = rho * ux;
    U[2 * nS + s] = rho * uy;
    U[3 * nS + s] = rho * uz;
    U[4 * nS + s] = rho * (e + 0.5 * (ux * ux + uy * uy + uz * uz));
#pragma unroll
    for (int k = 0; k < NS; ++k) U[(5 + k) * nS + s] = rho * Yk[k];
  }
}

// Periodic ghost fill.  Work items are chunks of the ghost cells of a box,
// enumerated as the two z slabs, then the y slabs of the interior z range,
// then the x slabs of the interior (y, z) range.
template <int NCOMP>
__global__ __launch_bounds__(256) void k_ghost(const BoxDev *__restrict__ boxes,
                                               const Item *__restrict__ items, int nitems,
                                               FRef Uref) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    long long g = (long long)w.x0 + threadIdx.x;
    const long long A = 2LL * NSDC_NG * b.sy * b.sx;
    const long long B = (long long)b.nz * 2 * NSDC_NG * b.sx;
    const long long C = (long long)b.nz * b.ny * 2 * NSDC_NG;
    if (g >= A + B + C) continue;
    int x, y, z;
    if (g < A) {
      const int zz = (int)(g / ((long long)b.sy * b.sx));
      const long long r = g % ((long long)b.sy * b.sx);
      y = (int)(r / b.sx);
      x = (int)(r % b.sx);
      z = zz < NSDC_NG ? zz : b.nz + zz;
    } else if (g < A + B) {
      g -= A;
      z = NSDC_NG + (int)(g / (2LL * NSDC_NG * b.sx));
      const long long r = g % (2LL * NSDC_NG * b.sx);
      const int yy = (int)(r / b.sx);
      x = (int)(r % b.sx);
      y = yy < NSDC_NG ? yy : b.ny + yy;
    } else {
      g -= A + B;
      z = NSDC_NG + (int)(g / (2LL * NSDC_NG * b.ny));
      const long long r = g % (2LL * NSDC_NG * b.ny);
      y = NSDC_NG + (int)(r / (2 * NSDC_NG));
      const int xx = (int)(r % (2 * NSDC_NG));
      x = xx < NSDC_NG ? xx : b.nx + xx;
    }
    const int xs = ((x - NSDC_NG) % b.nx + b.nx) % b.nx + NSDC_NG;
    const int ys = ((y - NSDC_NG) % b.ny + b.ny) % b.ny + NSDC_NG;
    const int zs = ((z - NSDC_NG) % b.nz + b.nz) % b.nz + NSDC_NG;
    const long long nS = (long long)b.sx * b.sy * b.sz;
    const long long dst = ((long long)z * b.sy + y) * b.sx + x;
    const long long src = ((long long)zs * b.sy + ys) * b.sx + xs;
    double *U = Uref.get(w.box, b.offS * NCOMP);
#pragma unroll 4
    for (int q = 0; q < NCOMP; ++q) U[q * nS + dst] = U[q * nS + src];
  }
}

// out_mode: 0 leave the right-hand side alone, 1 zero it, 2 chemistry source
template <int NS>
__global__ __launch_bounds__(256) void k_prims(const BoxDev *__restrict__ boxes,
                                               const Item *__restrict__ items, int nitems,
                                               TileShape ts, FRef Uref, double *__restrict__ Pbase,
                                               FRef Fout, int out_mode,
                                               const DevMech *__restrict__ m, int *err) {
  using L = Layout<NS>;
  constexpr int NU = L::NU, NP = L::NP;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int x, y, z;
    tile_cell(w, ts, x, y, z);
    if (x >= b.sx || y >= b.sy || z >= b.sz) continue;
    const long long nS = (long long)b.sx * b.sy * b.sz;
    const long long s = ((long long)z * b.sy + y) * b.sx + x;
    const double *U = Uref.get(w.box, b.offS * NU);
    double *P = Pbase + b.offS * NP;
    double Uc[NU];
#pragma unroll
    for (int q = 0; q < NU; ++q) Uc[q] = U[q * nS + s];
    double rho, u[3], Y[NS], T;
    const int e = cell_state<NS>(m, Uc, rho, u, Y, T);
    if (e) atomicOr(err, e);
    const double invT = 1.0 / T;
    double sumYW = 0.0, cp = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      sumYW += Y[k] * m->invW[k];
      cp += Y[k] * m->Rk[k] * cp_R(m, k, T);
    }
    const double Wbar = 1.0 / sumYW;
    const double pr = rho * RU * T * sumYW;
    const double mu = m->mu_ref * pow(T * m->inv_Tref, m->mu_exp);
    const double lam = mu * cp * m->inv_Pr;
    P[L::PU * nS + s] = u[0];
    P[L::PV * nS + s] = u[1];
    P[L::PW * nS + s] = u[2];
    P[L::PT * nS + s] = T;
    P[L::PP * nS + s] = pr;
    P[L::PMU * nS + s] = mu;
    P[L::PLAM * nS + s] = lam;
    P[L::PRD * nS + s] = lam / cp;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      P[(L::PY + k) * nS + s] = Y[k];
      P[(L::PX + k) * nS + s] = Y[k] * Wbar * m->invW[k];
      P[(L::PH + k) * nS + s] = m->Rk[k] * T * h_RT(m, k, T, invT);
    }
    if (out_mode == 0) continue;
    const int xi = x - NSDC_NG, yi = y - NSDC_NG, zi = z - NSDC_NG;
    if (xi < 0 || yi < 0 || zi < 0 || xi >= b.nx || yi >= b.ny || zi >= b.nz) continue;
    const long long nI = (long long)b.nx * b.ny * b.nz;
    const long long i = ((long long)zi * b.ny + yi) * b.nx + xi;
    double *F = Fout.get(w.box, b.offI * NU);
#pragma unroll
    for (int q = 0; q < 5; ++q) F[q * nI + i] = 0.0;
    if (out_mode == 2) {
      double wd[NS];
      production<NS>(m, rho, T, Y, wd);
#pragma unroll
      for (int k = 0; k < NS; ++k) F[(5 + k) * nI + i] = wd[k];
    } else {
#pragma unroll
      for (int k = 0; k < NS; ++k) F[(5 + k) * nI + i] = 0.0;
    }
  }
}

// Velocity gradient G[3 j + i] = D_j u_i at every stored cell whose
// j-coordinate is interior (the only places it is read).
template <int NS>
__global__ __launch_bounds__(256) void k_vgrad(const BoxDev *__restrict__ boxes,
                                               const Item *__restrict__ items, int nitems,
                                               TileShape ts, const double *__restrict__ Pbase,
                                               double *__restrict__ Gbase) {
  using L = Layout<NS>;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int x, y, z;
    tile_cell(w, ts, x, y, z);
    if (x >= b.sx || y >= b.sy || z >= b.sz) continue;
    const long long nS = (long long)b.sx * b.sy * b.sz;
    const long long s = ((long long)z * b.sy + y) * b.sx + x;
    const double *P = Pbase + b.offS * L::NP;
    double *G = Gbase + b.offS * 9;
    const int c[3] = {x, y, z};
    const int n[3] = {b.nx, b.ny, b.nz};
    const long long st[3] = {1, b.sx, (long long)b.sx * b.sy};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if (c[j] < NSDC_NG || c[j] >= n[j] + NSDC_NG) continue;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double *f = P + (L::PU + i) * nS + s;
        double v[9];
#pragma unroll
        for (int o = 0; o < 9; ++o) v[o] = f[(o - 4) * st[j]];
        G[(3 * j + i) * nS + s] = d1(v, b.idx[j]);
      }
    }
  }
}

// Row sums of the narrow-stencil matrix for one field at the two faces of
// the centre cell: Rp[r] = sum_c M[r][c] u[1+c] (face i+1/2), Rm[r] with
// u[c] (face i-1/2); the zero corners of M are skipped.
struct Rows {
  double p[8], m[8];
};
__device__ __forceinline__ void rows(const DevMech *__restrict__ mm, const double *u, Rows &R) {
  const int lo[8] = {0, 0, 0, 0, 0, 1, 2, 3};
  const int hi[8] = {4, 5, 6, 7, 7, 7, 7, 7};
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    double sp = 0.0, sm = 0.0;
#pragma unroll
    for (int c = lo[r]; c <= hi[r]; ++c) {
      const double Mrc = mm->M[r][c];
      sp += Mrc * u[1 + c];
      sm += Mrc * u[c];
    }
    R.p[r] = sp;
    R.m[r] = sm;
  }
}
// (H_{i+1/2} - H_{i-1/2}) / dx^2 with H = sum_m a_{i+m} (row sum m)
__device__ __forceinline__ double narrow(const double *a, const Rows &R, double idx2) {
  double hp = 0.0, hm = 0.0;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    hp += a[1 + r] * R.p[r];
    hm += a[r] * R.m[r];
  }
  return (hp - hm) * idx2;
}

template <int NS, int D>
__global__ __launch_bounds__(256) void k_dir(const BoxDev *__restrict__ boxes,
                                             const Item *__restrict__ items, int nitems,
                                             TileShape ts, FRef Uref,
                                             const double *__restrict__ Pbase,
                                             const double *__restrict__ Gbase, FRef Fout,
                                             unsigned parts, const DevMech *__restrict__ m) {
  using L = Layout<NS>;
  constexpr int NU = L::NU, NP = L::NP;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int x, y, z;
    tile_cell(w, ts, x, y, z);
    if (x >= b.nx || y >= b.ny || z >= b.nz) continue;
    const long long nS = (long long)b.sx * b.sy * b.sz;
    const long long nI = (long long)b.nx * b.ny * b.nz;
    const long long s = ((long long)(z + NSDC_NG) * b.sy + (y + NSDC_NG)) * b.sx + (x + NSDC_NG);
    const long long i = ((long long)z * b.ny + y) * b.nx + x;
    const long long st = D == 0 ? 1 : (D == 1 ? (long long)b.sx : (long long)b.sx * b.sy);
    const double *U = Uref.get(w.box, b.offS * NU);
    const double *P = Pbase + b.offS * NP;
    const double *G = Gbase + b.offS * 9;
    double *F = Fout.get(w.box, b.offI * NU);
    const double idx = b.idx[D], idx2 = b.idx2[D];
    double acc[NU];
#pragma unroll
    for (int q = 0; q < NU; ++q) acc[q] = 0.0;
    auto line = [&](const double *f, double *v) {
#pragma unroll
      for (int o = 0; o < 9; ++o) v[o] = f[s + (o - 4) * st];
    };
    double ud[9], pp[9];
    line(P + (L::PU + D) * nS, ud);
    line(P + L::PP * nS, pp);

    if (parts & 1) {  // convective terms -D_D(F_D(U))
      double f[9], Uq[9];
      line(U + (1 + D) * nS, f);
      acc[0] -= d1(f, idx);
#pragma unroll
      for (int ic = 0; ic < 3; ++ic) {
        line(U + (1 + ic) * nS, Uq);
#pragma unroll
        for (int o = 0; o < 9; ++o) f[o] = Uq[o] * ud[o] + (ic == D ? pp[o] : 0.0);
        acc[1 + ic] -= d1(f, idx);
      }
      line(U + 4 * nS, Uq);
#pragma unroll
      for (int o = 0; o < 9; ++o) f[o] = (Uq[o] + pp[o]) * ud[o];
      acc[4] -= d1(f, idx);
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        line(U + (5 + k) * nS, Uq);
#pragma unroll
        for (int o = 0; o < 9; ++o) f[o] = Uq[o] * ud[o];
        acc[5 + k] -= d1(f, idx);
      }
    }

    if (parts & 2) {  // diffusive terms
      const double bulk = m->bulk;
      double mu[9], a[9], v[9], vel[3][9];
      Rows R;
      line(P + L::PMU * nS, mu);
#pragma unroll
      for (int c = 0; c < 3; ++c) line(P + (L::PU + c) * nS, vel[c]);
      // viscous momentum: L_D(a, u_i), a = 4/3 mu + xi along i = D, mu otherwise
#pragma unroll
      for (int ic = 0; ic < 3; ++ic) {
#pragma unroll
        for (int o = 0; o < 9; ++o) a[o] = ic == D ? (4.0 / 3.0 + bulk) * mu[o] : mu[o];
        rows(m, vel[ic], R);
        acc[1 + ic] += narrow(a, R, idx2);
      }
      // heat conduction L_D(lambda, T)
      line(P + L::PLAM * nS, a);
      line(P + L::PT * nS, v);
      rows(m, v, R);
      acc[4] += narrow(a, R, idx2);
      // viscous work: L_D(mu, |u|^2/2) + L_D(mu/3 + xi, u_D^2/2)
#pragma unroll
      for (int o = 0; o < 9; ++o)
        v[o] = 0.5 * (vel[0][o] * vel[0][o] + vel[1][o] * vel[1][o] + vel[2][o] * vel[2][o]);
      rows(m, v, R);
      acc[4] += narrow(mu, R, idx2);
#pragma unroll
      for (int o = 0; o < 9; ++o) {
        v[o] = 0.5 * ud[o] * ud[o];
        a[o] = (1.0 / 3.0 + bulk) * mu[o];
      }
      rows(m, v, R);
      acc[4] += narrow(a, R, idx2);
      // mixed terms: D_D(mu D_i u_D) (i != D), D_D((xi - 2/3 mu) sum_{j!=D} D_j u_j),
      // D_D(mu sum_{j!=D} u_j D_j u_D + (xi - 2/3 mu) u_D sum_{j!=D} D_j u_j)
      {
        constexpr int J1 = D == 0 ? 1 : 0, J2 = D == 2 ? 1 : 2;
        double g1D[9], g2D[9], dsum[9], f[9];
        line(G + (3 * J1 + D) * nS, g1D);
        line(G + (3 * J2 + D) * nS, g2D);
        line(G + (3 * J1 + J1) * nS, a);
        line(G + (3 * J2 + J2) * nS, v);
#pragma unroll
        for (int o = 0; o < 9; ++o) dsum[o] = a[o] + v[o];
#pragma unroll
        for (int o = 0; o < 9; ++o) f[o] = mu[o] * g1D[o];
        acc[1 + J1] += d1(f, idx);
#pragma unroll
        for (int o = 0; o < 9; ++o) f[o] = mu[o] * g2D[o];
        acc[1 + J2] += d1(f, idx);
#pragma unroll
        for (int o = 0; o < 9; ++o) f[o] = (bulk - 2.0 / 3.0) * mu[o] * dsum[o];
        acc[1 + D] += d1(f, idx);
#pragma unroll
        for (int o = 0; o < 9; ++o)
          f[o] = mu[o] * (vel[J1][o] * g1D[o] + vel[J2][o] * g2D[o]) +
                 (bulk - 2.0 / 3.0) * mu[o] * vel[D][o] * dsum[o];
        acc[4] += d1(f, idx);
      }
      // species diffusion with the correction velocity (direction-D share)
      {
        double rd[9], ep[9], Rpp[8], Rpm[8];
        line(P + L::PRD * nS, rd);
        rows(m, pp, R);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          Rpp[r] = R.p[r];
          Rpm[r] = R.m[r];
        }
        const double Dp = d1(pp, idx);
        const double ip = 1.0 / pp[4];
#pragma unroll
        for (int o = 0; o < 9; ++o) ep[o] = 0.0;
        double divVc = 0.0, Vc = 0.0;
        double DY[NS], DhY[NS], Yc[NS], hc[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const double iLe = m->invLe[k];
          double X[9], Yv[9], h[9], ad[9], ap[9], f[9];
          line(P + (L::PX + k) * nS, X);
          line(P + (L::PY + k) * nS, Yv);
          line(P + (L::PH + k) * nS, h);
#pragma unroll
          for (int o = 0; o < 9; ++o) {
            ad[o] = rd[o] * iLe;
            ap[o] = ad[o] * (X[o] - Yv[o]) / pp[o];
            ep[o] += ap[o] * h[o];
          }
          rows(m, X, R);
          const double Lx = narrow(ad, R, idx2);
          Rows Rp;
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            Rp.p[r] = Rpp[r];
            Rp.m[r] = Rpm[r];
          }
          const double Lp = narrow(ap, Rp, idx2);
          acc[5 + k] += Lx + Lp;
          divVc -= Lx + Lp;
#pragma unroll
          for (int o = 0; o < 9; ++o) f[o] = ad[o] * h[o];
          acc[4] += narrow(f, R, idx2);
          Vc -= ad[4] * (d1(X, idx) + (X[4] - Yv[4]) * Dp * ip);
          DY[k] = d1(Yv, idx);
#pragma unroll
          for (int o = 0; o < 9; ++o) f[o] = h[o] * Yv[o];
          DhY[k] = d1(f, idx);
          Yc[k] = Yv[4];
          hc[k] = h[4];
        }
        {
          Rows Rp;
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            Rp.p[r] = Rpp[r];
            Rp.m[r] = Rpm[r];
          }
          acc[4] += narrow(ep, Rp, idx2);
        }
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          acc[5 + k] += Yc[k] * divVc + Vc * DY[k];
          acc[4] += hc[k] * Yc[k] * divVc + Vc * DhY[k];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NU; ++q) F[q * nI + i] += acc[q];
  }
}

// Chemistry source of the current state on the interior (the fine component
// f2 of the multirate scheme): F2[k] = rho omega_k(U).
template <int NS>
__global__ __launch_bounds__(256) void k_chem(const BoxDev *__restrict__ boxes,
                                              const Item *__restrict__ items, int nitems,
                                              TileShape ts, FRef Uref, double *__restrict__ F2base,
                                              const DevMech *__restrict__ m, int *err) {
  constexpr int NU = 5 + NS;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int x, y, z;
    tile_cell(w, ts, x, y, z);
    if (x >= b.nx || y >= b.ny || z >= b.nz) continue;
    const long long nS = (long long)b.sx * b.sy * b.sz, nI = (long long)b.nx * b.ny * b.nz;
    const long long s = ((long long)(z + NSDC_NG) * b.sy + (y + NSDC_NG)) * b.sx + (x + NSDC_NG);
    const long long i = ((long long)z * b.ny + y) * b.nx + x;
    const double *U = Uref.get(w.box, b.offS * NU);
    double *F2 = F2base + b.offI * NS;
    double Uc[NU];
#pragma unroll
    for (int q = 0; q < NU; ++q) Uc[q] = U[q * nS + s];
    double rho, u[3], Y[NS], T, wd[NS];
    const int e = cell_state<NS>(m, Uc, rho, u, Y, T);
    if (e) atomicOr(err, e);
    production<NS>(m, rho, T, Y, wd);
#pragma unroll
    for (int k = 0; k < NS; ++k) F2[k * nI + i] = wd[k];
  }
}

// Single-rate SDC node update (eq. expsdc):
//   U_{m+1} = U_m + dtau_m (F^{k+1}_m - F^k_m) + dt sum_j S_{mj} F^k_j


template <int NS>
__global__ __launch_bounds__(256) void k_sdc_node(const BoxDev *__restrict__ boxes,
                                                  const Item *__restrict__ items, int nitems,
                                                  TileShape ts, FRef Ucur, FRef Unext,
                                                  NodeArgs a) {
  constexpr int NU = 5 + NS;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int x, y, z;
    tile_cell(w, ts, x, y, z);
    if (x >= b.nx || y >= b.ny || z >= b.nz) continue;
    const long long nS = (long long)b.sx * b.sy * b.sz, nI = (long long)b.nx * b.ny * b.nz;
    const long long s = ((long long)(z + NSDC_NG) * b.sy + (y + NSDC_NG)) * b.sx + (x + NSDC_NG);
    const long long i = ((long long)z * b.ny + y) * b.nx + x;
    const long long oI = b.offI * NU;
    const double *Uc = Ucur.get(w.box, b.offS * NU);
    double *Un = Unext.get(w.box, b.offS * NU);
    for (int q = 0; q < NU; ++q) {
      const long long qi = oI + q * nI + i;
      double sf = 0.0;
      for (int j = 0; j < a.nnodes; ++j) sf += a.S[j] * a.Fold[j][qi];
      Un[q * nS + s] = Uc[q * nS + s] + a.dtau * (a.Fnew_m[qi] - a.Fold_m[qi]) + a.dt * sf;
    }
  }
}

// One coarse interval of the multirate sweep, mode 1 (eq. mrupdate), all
// fine sub-steps of the interval for one cell in registers:
//   U_{q+1} = U_q + dtau_q [f1(U^{k+1}_p) - f1(U^k_p)] + dtau_q [f2(U^{k+1}_q) - f2(U^k_q)]
//             + dt S22_q . F2^k + dt S21_q . F1^k,
// with f2 the chemistry (species components only) evaluated here.
template <int NS>
__global__ __launch_bounds__(256) void k_mr_fine(const BoxDev *__restrict__ boxes,
                                                 const Item *__restrict__ items, int nitems,
                                                 TileShape ts, FRef Uin, FRef Uout,
                                                 const FineCoef *__restrict__ fc, FinePtrs fp,
                                                 const DevMech *__restrict__ m, int *err) {
  constexpr int NU = 5 + NS;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int x, y, z;
    tile_cell(w, ts, x, y, z);
    if (x >= b.nx || y >= b.ny || z >= b.nz) continue;
    const long long nS = (long long)b.sx * b.sy * b.sz, nI = (long long)b.nx * b.ny * b.nz;
    const long long s = ((long long)(z + NSDC_NG) * b.sy + (y + NSDC_NG)) * b.sx + (x + NSDC_NG);
    const long long i = ((long long)z * b.ny + y) * b.nx + x;
    const long long o1 = b.offI * NU, o2 = b.offI * NS;
    const double *Ui = Uin.get(w.box, b.offS * NU);
    double *Uo = Uout.get(w.box, b.offS * NU);
    double Uc[NU];
#pragma unroll
    for (int q = 0; q < NU; ++q) Uc[q] = Ui[q * nS + s];
    const int n1 = fc->n1, nq = fc->nq;
    const double dt = fp.dt;
    int errs = 0;
    for (int qq = 0; qq < nq; ++qq) {
      double f2[NS];
      if (qq == 0 && fp.q0_known) {
#pragma unroll
        for (int k = 0; k < NS; ++k) f2[k] = fp.F2old[0][o2 + k * nI + i];
      } else {
        double rho, u[3], Y[NS], T;
        errs |= cell_state<NS>(m, Uc, rho, u, Y, T);
        production<NS>(m, rho, T, Y, f2);
#pragma unroll
        for (int k = 0; k < NS; ++k) fp.F2new[qq][o2 + k * nI + i] = f2[k];
      }
      const double dtq = fc->dtq[qq] * dt;
#pragma unroll
      for (int q = 0; q < NU; ++q) {
        const long long qi = o1 + q * nI + i;
        double s21 = 0.0;
        for (int j = 0; j < n1; ++j) s21 += fc->S21[qq][j] * fp.F1old[j][qi];
        double du = dtq * (fp.F1new_p[qi] - fp.F1old_p[qi]) + dt * s21;
        if (q >= 5) {
          const int k = q - 5;
          const long long ki = o2 + k * nI + i;
          double s22 = 0.0;
          for (int j = 0; j <= nq; ++j) s22 += fc->S22[qq][j] * fp.F2old[j][ki];
          du += dtq * (f2[k] - fp.F2old[qq][ki]) + dt * s22;
        }
        Uc[q] += du;
      }
    }
    if (fp.eval_last) {
      double rho, u[3], Y[NS], T, f2[NS];
      errs |= cell_state<NS>(m, Uc, rho, u, Y, T);
      production<NS>(m, rho, T, Y, f2);
#pragma unroll
      for (int k = 0; k < NS; ++k) fp.F2new[nq][o2 + k * nI + i] = f2[k];
    }
    if (errs) atomicOr(err, errs);
#pragma unroll
    for (int q = 0; q < NU; ++q) Uo[q * nS + s] = Uc[q];
  }
}

}  // namespace nsdc

// ------------------------------------------------------------ launchers
#include "launch.h"

namespace nsdc {

static inline int grid_for(int nitems, int cap) { return nitems < cap ? (nitems > 0 ? nitems : 1) : cap; }

template <int NS>
struct Launch {
  static void prim_to_cons(const LaunchCtx &c, const double *p, const double *T, const double *Y,
                           const double *u, FRef U) {
    prof_begin(c.prof, K_PRIM_TO_CONS, c.stream);
    hipLaunchKernelGGL(k_prim_to_cons<NS>, dim3(grid_for(c.nI, c.cap)), dim3(c.tsI.tx * c.tsI.ty * c.tsI.tz), 0,
                       c.stream, c.boxes, c.itemsI, c.nI, c.tsI, p, T, Y, u, U, c.mech);
    prof_end(c.prof, K_PRIM_TO_CONS, c.stream);
  }
  static void ghost(const LaunchCtx &c, FRef U) {
    prof_begin(c.prof, K_GHOST, c.stream);
    hipLaunchKernelGGL(k_ghost<5 + NS>, dim3(grid_for(c.nG, c.cap)), dim3(256), 0, c.stream, c.boxes,
                       c.itemsG, c.nG, U);
    prof_end(c.prof, K_GHOST, c.stream);
  }
  static void prims(const LaunchCtx &c, FRef U, double *P, FRef F, int out_mode) {
    prof_begin(c.prof, K_PRIMS, c.stream);
    hipLaunchKernelGGL(k_prims<NS>, dim3(grid_for(c.nS, c.cap)), dim3(c.tsS.tx * c.tsS.ty * c.tsS.tz), 0,
                       c.stream, c.boxes, c.itemsS, c.nS, c.tsS, U, P, F, out_mode, c.mech, c.err);
    prof_end(c.prof, K_PRIMS, c.stream);
  }
  static void vgrad(const LaunchCtx &c, const double *P, double *G) {
    prof_begin(c.prof, K_VGRAD, c.stream);
    hipLaunchKernelGGL(k_vgrad<NS>, dim3(grid_for(c.nS, c.cap)), dim3(c.tsS.tx * c.tsS.ty * c.tsS.tz), 0,
                       c.stream, c.boxes, c.itemsS, c.nS, c.tsS, P, G);
    prof_end(c.prof, K_VGRAD, c.stream);
  }
  static void dir(const LaunchCtx &c, int d, FRef U, const double *P, const double *G, FRef F,
                  unsigned parts) {
    const dim3 grid(grid_for(c.nI, c.cap)), block(c.tsI.tx * c.tsI.ty * c.tsI.tz);
    prof_begin(c.prof, K_DIR_X + d, c.stream);
    if (d == 0)
      hipLaunchKernelGGL((k_dir<NS, 0>), grid, block, 0, c.stream, c.boxes, c.itemsI, c.nI, c.tsI, U, P, G, F,
                         parts, c.mech);
    else if (d == 1)
      hipLaunchKernelGGL((k_dir<NS, 1>), grid, block, 0, c.stream, c.boxes, c.itemsI, c.nI, c.tsI, U, P, G, F,
                         parts, c.mech);
    else
      hipLaunchKernelGGL((k_dir<NS, 2>), grid, block, 0, c.stream, c.boxes, c.itemsI, c.nI, c.tsI, U, P, G, F,
                         parts, c.mech);
    prof_end(c.prof, K_DIR_X + d, c.stream);
  }
  static void chem(const LaunchCtx &c, FRef U, double *F2) {
    prof_begin(c.prof, K_CHEM, c.stream);
    hipLaunchKernelGGL(k_chem<NS>, dim3(grid_for(c.nI, c.cap)), dim3(c.tsI.tx * c.tsI.ty * c.tsI.tz), 0,
                       c.stream, c.boxes, c.itemsI, c.nI, c.tsI, U, F2, c.mech, c.err);
    prof_end(c.prof, K_CHEM, c.stream);
  }
  static void sdc_node(const LaunchCtx &c, FRef Ucur, FRef Unext, const NodeArgs &a) {
    prof_begin(c.prof, K_SDC_NODE, c.stream);
    hipLaunchKernelGGL(k_sdc_node<NS>, dim3(grid_for(c.nI, c.cap)), dim3(c.tsI.tx * c.tsI.ty * c.tsI.tz), 0,
                       c.stream, c.boxes, c.itemsI, c.nI, c.tsI, Ucur, Unext, a);
    prof_end(c.prof, K_SDC_NODE, c.stream);
  }
  static void mr_fine(const LaunchCtx &c, FRef Uin, FRef Uout, const FineCoef *fc,
                      const FinePtrs &fp) {
    prof_begin(c.prof, K_MR_FINE, c.stream);
    hipLaunchKernelGGL(k_mr_fine<NS>, dim3(grid_for(c.nI, c.cap)), dim3(c.tsI.tx * c.tsI.ty * c.tsI.tz), 0,
                       c.stream, c.boxes, c.itemsI, c.nI, c.tsI, Uin, Uout, fc, fp, c.mech, c.err);
    prof_end(c.prof, K_MR_FINE, c.stream);
  }
};

}  // namespace nsdc

namespace nsdc {
template <int NS>
static const Ops make_ops() {
  Ops o;
  o.ns = NS;
  o.prim_to_cons = &Launch<NS>::prim_to_cons;
  o.ghost = &Launch<NS>::ghost;
  o.prims = &Launch<NS>::prims;
  o.vgrad = &Launch<NS>::vgrad;
  o.dir = &Launch<NS>::dir;
  o.chem = &Launch<NS>::chem;
  o.sdc_node = &Launch<NS>::sdc_node;
  o.mr_fine = &Launch<NS>::mr_fine;
  return o;
}
static const Ops OPS9 = make_ops<9>();
static const Ops OPS21 = make_ops<21>();

const Ops *ops_for(int ns) {
  switch (ns) {
    case 9: return &OPS9;
    case 21: return &OPS21;
    default: return nullptr;
  }
}
}  // namespace nsdc
