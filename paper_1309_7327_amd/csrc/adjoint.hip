// Device kernels of the vector-Jacobian product of the right-hand side (the
// adjoint of eq. cns as discretised in Section 2.2), FP64, gfx950.
//
// Given a cotangent vbar of dU/dt on the interior, the product
// Ubar = (d rhs / dU)^T vbar is formed stage by stage in reverse:
//   k_adj_coef<D>  per output cell, the sums over species that the
//                  transposed direction-D terms need (div V_c, V_c, their
//                  adjoints, D p / p)
//   k_adj_g1..g3   transpose of every term that differentiates along D, as a
//                  gather: a thread takes one sample cell and collects the
//                  contributions of the nine output cells whose lines
//                  contain it (convective, viscous, mixed and heat terms in
//                  g1; species diffusion and correction velocity in g2, g3)
//   k_chem_adj     transpose of the chemistry source; also the products
//                  with respect to ln A_j, reduced per workgroup in a fixed
//                  order (wave butterflies, then the waves in index order)
//   k_vgrad_adj    transpose of the velocity gradient G = D_j u_i (a gather)
//   k_prims_adj    transpose of the conserved -> primitive map at every
//                  stored cell, with the implicit-function derivative of the
//                  Newton temperature, dT = (de - sum_k e_k dY_k) / c_v
//   k_fold         ghost cells are periodic copies: the adjoint of a ghost
//                  cell is added to its interior source (a gather over the
//                  periodic images of each interior cell)
//   k_lnA_reduce   sums the per-workgroup ln A partials in index order
#include <math.h>

#include "adjoint.h"
#include "physics.h"

namespace nsdc {

namespace {
// eighth-order first-derivative weights of the nine samples (times 1/dx)
__device__ __forceinline__ void d1w(double idx, double *w) {
  w[4] = 0.0;
  w[5] = C1 * idx; w[3] = -w[5];
  w[6] = C2 * idx; w[2] = -w[6];
  w[7] = C3 * idx; w[1] = -w[7];
  w[8] = C4 * idx; w[0] = -w[8];
}

// bt = B^T a (B banded: column c spans rows c-4..c+4)
template <bool FIXED>
__device__ __forceinline__ void btvec(const DevMech *__restrict__ m, const double *a, double *bt) {
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    double acc = 0.0;
#pragma unroll
    for (int o = (c > 4 ? c - 4 : 0); o <= (c < 4 ? c + 4 : 8); ++o)
      acc += (FIXED ? SMC_B.v[o][c] : m->B[o][c]) * a[o];
    bt[c] = acc;
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
}  // namespace

// Zero n doubles.
__global__ __launch_bounds__(256) void k_fill0(double *__restrict__ p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// Y_t[i] += c_t X[i], t < nt (flat arrays of n doubles).
__global__ __launch_bounds__(256) void k_axpy_multi(const double *__restrict__ X, AxpyArgs a, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double x = X[i];
    for (int t = 0; t < a.nt; ++t) a.Y[t][i] += a.c[t] * x;
  }
}

// Y[i] = sum_t c_t X_t[i] (flat arrays of n doubles).
__global__ __launch_bounds__(256) void k_lincomb(LincombArgs a, double *__restrict__ Y, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int t = 0; t < a.nt; ++t) s += a.c[t] * a.X[t][i];
    Y[i] = s;
  }
}

// ------------------------------------------------- direction adjoint (gather)
// For direction D, output cell i and sample o of its nine-point line, the
// forward terms are sums over o of (per-output-cell factor) x (sample
// value), or products with rows of B.  The adjoint of a field at a sample
// cell s collects the contributions of the nine output cells j_o = s - (o-4)
// e_D whose lines contain s (s is their sample o):
//   sum_o f(j_o) dw_o                       first-derivative terms
//   sum_o f(j_o) sum_c B_oc W[s + c - o]     the coefficient side of L (brow)
//   sum_o f(j_o) sum_c B_co W[s + c - o]     the field side of L (bcol)
// with W a 17-sample window of a primitive field around s.  The factors
// that need a sum over all species of an output cell (div V_c, V_c, their
// adjoints, D p / p) come from a per-output-cell pass (k_adj_coef).  Every
// thread writes only its own cell: no atomics, no phases.

// coefficient table per output cell and direction
enum { CF_DIVVC = 0, CF_VC, CF_DIVVCB, CF_VCB, CF_DPP, CF_DPPB, CF_RDSELF, CF_N };

namespace {
template <bool FIXED>
__device__ __forceinline__ double bmat(const DevMech *__restrict__ m, int o, int c) {
  return FIXED ? SMC_B.v[o][c] : m->B[o][c];
}
// row o of B against the window (W[8] = the sample cell)
template <bool FIXED>
__device__ __forceinline__ double brow(const DevMech *__restrict__ m, const double *W, int o) {
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < 9; ++c)
    if (c >= o - 4 && c <= o + 4) acc += bmat<FIXED>(m, o, c) * W[c - o + 8];
  return acc;
}
// column o of B against the window
template <bool FIXED>
__device__ __forceinline__ double bcol(const DevMech *__restrict__ m, const double *W, int o) {
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < 9; ++c)
    if (c >= o - 4 && c <= o + 4) acc += bmat<FIXED>(m, c, o) * W[c - o + 8];
  return acc;
}

// Geometry of a gather thread: stored cell s whose two transverse
// coordinates are interior; output cell j_o has interior D-coordinate
// cd - o (cd = stored D-coordinate of s).  Per-lane indices are 32-bit
// (a box has < 2^28 stored cells); field bases stay 64-bit and uniform.
template <int D>
struct Gather {
  long long nS, nI;
  int s, st, ibase, sI, cd, nD, lo, hi;
  bool ok;
  __device__ Gather(const BoxDev &b, int x, int y, int z) {
    const int c[3] = {x, y, z}, n[3] = {b.nx, b.ny, b.nz};
    ok = x < b.sx && y < b.sy && z < b.sz;
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (d != D && (c[d] < NSDC_NG || c[d] >= n[d] + NSDC_NG)) ok = false;
    nS = (long long)b.sx * b.sy * b.sz;
    nI = (long long)b.nx * b.ny * b.nz;
    s = (z * b.sy + y) * b.sx + x;
    st = D == 0 ? 1 : (D == 1 ? b.sx : b.sx * b.sy);
    sI = D == 0 ? 1 : (D == 1 ? b.nx : b.nx * b.ny);
    cd = c[D];
    nD = n[D];
    const int xi = D == 0 ? 0 : x - NSDC_NG, yi = D == 1 ? 0 : y - NSDC_NG, zi = D == 2 ? 0 : z - NSDC_NG;
    ibase = (zi * b.ny + yi) * b.nx + xi;
    lo = s - cd * st;                              // stored D-coordinate 0
    hi = s + (nD + 2 * NSDC_NG - 1 - cd) * st;     // last stored D-coordinate
  }
  __device__ bool valid(int o) const { return cd - o >= 0 && cd - o < nD; }
  __device__ int j(int o) const { return ibase + (cd - o) * sI; }
  // interior field value at output cell j_o (0 where j_o is not a cell)
  __device__ double at(const double *f, int o) const { return valid(o) ? f[j(o)] : 0.0; }
  // 17-sample window of a stored field around s (clamped at the array ends;
  // clamped samples only meet the zero factors of absent output cells)
  __device__ void window(const double *f, double *W) const {
    int p = s - 8 * st;
#pragma unroll
    for (int mm = 0; mm < 17; ++mm, p += st) W[mm] = f[min(max(p, lo), hi)];
  }
};
}  // namespace

// Per output cell: the forward sums div V_c, V_c, their adjoints and the
// pressure-gradient factor of direction D (CF_* table, interior layout).
template <int NS, int D, bool FIXED>
__global__ __launch_bounds__(256) void k_adj_coef(const BoxDev *__restrict__ boxes,
                                                  const Item *__restrict__ items, int nitems, TileShape ts,
                                                  const double *__restrict__ Pbase,
                                                  const double *__restrict__ Vbase, double *__restrict__ coef,
                                                  const DevMech *__restrict__ m) {
  using L = Layout<NS>;
  constexpr int NU = L::NU, NP = L::NP;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int x, y, z;
    tile_cell(w, ts, x, y, z);
    if (x >= b.nx || y >= b.ny || z >= b.nz) continue;
    const long long nS = (long long)b.sx * b.sy * b.sz, nI = (long long)b.nx * b.ny * b.nz;
    const long long s = ((long long)(z + NSDC_NG) * b.sy + (y + NSDC_NG)) * b.sx + (x + NSDC_NG);
    const long long i = ((long long)z * b.ny + y) * b.nx + x;
    const long long st = D == 0 ? 1 : (D == 1 ? (long long)b.sx : (long long)b.sx * b.sy);
    const double *P = Pbase + b.offS * NP;
    const double *V = Vbase + b.offI * NU;
    double *C = coef + b.offI * CF_N;
    const double idx = b.idx[D], idx2 = b.idx2[D];
    auto line = [&](const double *f, double *v) {
#pragma unroll
      for (int o = 0; o < 9; ++o) v[o] = f[s + (o - 4) * st];
    };
    double rd[9], pp[9], Bp[9], wp[9];
    line(P + L::PRD * nS, rd);
    line(P + L::PP * nS, pp);
    bvec<FIXED>(m, pp, Bp);
#pragma unroll
    for (int o = 0; o < 9; ++o) wp[o] = rd[o] * Bp[o] / pp[o];
    const double Dpp = d1(pp, idx) / pp[4];
    const double rd4 = rd[4];
    const double vb4 = V[4 * nI + i];
    double divVc = 0.0, Vc = 0.0, divVcb = 0.0, Vcb = 0.0, S1 = 0.0, S2 = 0.0;
#pragma unroll 1
    for (int k = 0; k < NS; ++k) {
      const double iLe = m->invLe[k];
      const double vbk = V[(5 + k) * nI + i];
      double X9[9], Y9[9], h9[9], v[9];
      line(P + (L::PX + k) * nS, X9);
      line(P + (L::PY + k) * nS, Y9);
      line(P + (L::PH + k) * nS, h9);
      bvec<FIXED>(m, X9, v);
      double Lxp = 0.0;
#pragma unroll
      for (int o = 0; o < 9; ++o) Lxp += rd[o] * v[o] + (X9[o] - Y9[o]) * wp[o];
      divVc -= iLe * Lxp * idx2;
      const double dXY4 = X9[4] - Y9[4];
      const double sv = iLe * (d1(X9, idx) + dXY4 * Dpp);
      Vc -= rd4 * sv;
      S1 += sv;
      S2 += iLe * dXY4;
      divVcb += (vbk + vb4 * h9[4]) * Y9[4];
      Vcb += vbk * d1(Y9, idx) + vb4 * d1p(h9, Y9, idx);
    }
    C[CF_DIVVC * nI + i] = divVc;
    C[CF_VC * nI + i] = Vc;
    C[CF_DIVVCB * nI + i] = divVcb;
    C[CF_VCB * nI + i] = Vcb;
    C[CF_DPP * nI + i] = Dpp;
    C[CF_DPPB * nI + i] = -Vcb * rd4 * S2;
    C[CF_RDSELF * nI + i] = -Vcb * S1;
  }
}

// Gather of the convective, viscous, mixed and heat-conduction terms of
// direction D into the state, velocity, pressure, viscosity, conductivity,
// temperature and velocity-gradient adjoints at sample cell s.
template <int NS, int D, bool FIXED>
__global__ __launch_bounds__(256) void k_adj_g1(const BoxDev *__restrict__ boxes,
                                                const Item *__restrict__ items, int nitems, TileShape ts,
                                                const double *__restrict__ Ubase,
                                                const double *__restrict__ Pbase,
                                                const double *__restrict__ Gbase,
                                                const double *__restrict__ Vbase, AdjBufs ab, unsigned parts,
                                                const DevMech *__restrict__ m) {
  using L = Layout<NS>;
  constexpr int NU = L::NU, NP = L::NP;
  constexpr int J1 = D == 0 ? 1 : 0, J2 = D == 2 ? 1 : 2;   // the two other directions
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int x, y, z;
    tile_cell(w, ts, x, y, z);
    const Gather<D> g(b, x, y, z);
    if (!g.ok) continue;
    const long long nS = g.nS, nI = g.nI, s = g.s;
    const double *U = Ubase + b.offS * NU;
    const double *P = Pbase + b.offS * NP;
    const double *G = Gbase + b.offS * 9;
    const double *V = Vbase + b.offI * NU;
    double *Ub = ab.Ub + b.offS * NU;
    double *Pb = ab.Pb + b.offS * NP;
    double *Gb = ab.Gb + b.offS * 9;
    const double idx = b.idx[D], idx2 = b.idx2[D];
    double dw[9];
    d1w(idx, dw);
    // cotangents of momentum and energy at the nine output cells
    double va[4][9];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int o = 0; o < 9; ++o) va[q][o] = g.at(V + (1 + q) * nI, o);
    double T[5];   // T_q = sum_o vbar_q(j_o) dw_o
    T[0] = 0.0;
#pragma unroll
    for (int o = 0; o < 9; ++o) T[0] += g.at(V, o) * dw[o];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      T[1 + q] = 0.0;
#pragma unroll
      for (int o = 0; o < 9; ++o) T[1 + q] += va[q][o] * dw[o];
    }
    double us[3];
#pragma unroll
    for (int ic = 0; ic < 3; ++ic) us[ic] = P[(L::PU + ic) * nS + s];
    const double ud = us[D], ps = P[L::PP * nS + s];
    double ub[3] = {0.0, 0.0, 0.0}, pb = 0.0;

    if (parts & 1) {  // -D_D(F_D(U))
      Ub[(1 + D) * nS + s] -= T[0];
#pragma unroll
      for (int ic = 0; ic < 3; ++ic) {
        Ub[(1 + ic) * nS + s] -= T[1 + ic] * ud;
        ub[D] -= T[1 + ic] * U[(1 + ic) * nS + s];
        if (ic == D) pb -= T[1 + D];
      }
      Ub[4 * nS + s] -= T[4] * ud;
      pb -= T[4] * ud;
      ub[D] -= T[4] * (U[4 * nS + s] + ps);
#pragma unroll 1
      for (int k = 0; k < NS; ++k) {
        double Tk = 0.0;
#pragma unroll
        for (int o = 0; o < 9; ++o) Tk += g.at(V + (5 + k) * nI, o) * dw[o];
        Ub[(5 + k) * nS + s] -= Tk * ud;
        ub[D] -= Tk * U[(5 + k) * nS + s];
      }
    }

    if (parts & 2) {
      const double bulk = m->bulk;
      const double lam2 = bulk - 2.0 / 3.0;
      const double ewD = 1.0 / 3.0 + bulk;
      double mub = 0.0, W[17], keW[17];
      // viscous stress L_D(mu, u_ic), viscous work L_D(mu/3 + xi, u_D^2/2)
      // and L_D(mu, |u|^2/2): field side at s ...
      g.window(P + L::PMU * nS, W);
      const double mus = W[8];
#pragma unroll
      for (int o = 0; o < 9; ++o) {
        const double beta = idx2 * bcol<FIXED>(m, W, o);
#pragma unroll
        for (int ic = 0; ic < 3; ++ic)
          ub[ic] += beta * (va[ic][o] * (ic == D ? 4.0 / 3.0 + bulk : 1.0) +
                            va[3][o] * (ic == D ? 1.0 + ewD : 1.0) * us[ic]);
      }
      // ... and coefficient side at s
#pragma unroll
      for (int mm = 0; mm < 17; ++mm) keW[mm] = 0.0;
#pragma unroll
      for (int ic = 0; ic < 3; ++ic) {
        g.window(P + (L::PU + ic) * nS, W);
#pragma unroll
        for (int o = 0; o < 9; ++o)
          mub += idx2 * va[ic][o] * (ic == D ? 4.0 / 3.0 + bulk : 1.0) * brow<FIXED>(m, W, o);
#pragma unroll
        for (int mm = 0; mm < 17; ++mm) {
          W[mm] = 0.5 * W[mm] * W[mm];
          keW[mm] += W[mm];
        }
        if (ic == D) {
#pragma unroll
          for (int o = 0; o < 9; ++o) mub += idx2 * va[3][o] * ewD * brow<FIXED>(m, W, o);
        }
      }
#pragma unroll
      for (int o = 0; o < 9; ++o) mub += idx2 * va[3][o] * brow<FIXED>(m, keW, o);
      // mixed terms D_D((xi - 2/3 mu) sum_{j != D} D_j u_j), D_D(mu D_ic u_D)
      // and their viscous work
      {
        const double gs = G[(3 * J1 + J1) * nS + s] + G[(3 * J2 + J2) * nS + s];
        const double Gm = T[1 + D] + us[D] * T[4];
        mub += lam2 * gs * Gm;
        Gb[(3 * J1 + J1) * nS + s] += lam2 * mus * Gm;
        Gb[(3 * J2 + J2) * nS + s] += lam2 * mus * Gm;
        ub[D] += lam2 * mus * gs * T[4];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int ic = e == 0 ? J1 : J2;
          const double gg = G[(3 * ic + D) * nS + s];
          const double Gi = T[1 + ic] + us[ic] * T[4];
          mub += gg * Gi;
          Gb[(3 * ic + D) * nS + s] += mus * Gi;
          ub[ic] += mus * gg * T[4];
        }
      }
      Pb[L::PMU * nS + s] += mub;
      // heat conduction L_D(lambda, T)
      {
        double lb = 0.0, tb = 0.0;
        g.window(P + L::PT * nS, W);
#pragma unroll
        for (int o = 0; o < 9; ++o) lb += va[3][o] * brow<FIXED>(m, W, o);
        g.window(P + L::PLAM * nS, W);
#pragma unroll
        for (int o = 0; o < 9; ++o) tb += va[3][o] * bcol<FIXED>(m, W, o);
        Pb[L::PLAM * nS + s] += idx2 * lb;
        Pb[L::PT * nS + s] += idx2 * tb;
      }
    }
#pragma unroll
    for (int ic = 0; ic < 3; ++ic) Pb[(L::PU + ic) * nS + s] += ub[ic];
    Pb[L::PP * nS + s] += pb;
  }
}

// Gather of the species diffusion and correction-velocity terms of
// direction D, in two kernels that each carry half of the state: g2 into
// the X_k, Y_k, h_k adjoints at s, g3 into the rho D and pressure adjoints.
template <int NS, int D, bool FIXED>
__global__ __launch_bounds__(256) void k_adj_g2(const BoxDev *__restrict__ boxes,
                                                const Item *__restrict__ items, int nitems, TileShape ts,
                                                const double *__restrict__ Pbase,
                                                const double *__restrict__ Vbase,
                                                const double *__restrict__ coef, AdjBufs ab,
                                                const DevMech *__restrict__ m) {
  using L = Layout<NS>;
  constexpr int NU = L::NU, NP = L::NP;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int x, y, z;
    tile_cell(w, ts, x, y, z);
    const Gather<D> g(b, x, y, z);
    if (!g.ok) continue;
    const long long nS = g.nS, nI = g.nI;
    const int s = g.s;
    const double *P = Pbase + b.offS * NP;
    const double *V = Vbase + b.offI * NU;
    const double *C = coef + b.offI * CF_N;
    double *Pb = ab.Pb + b.offS * NP;
    const double idx = b.idx[D], idx2 = b.idx2[D];
    double dw[9];
    d1w(idx, dw);
    double rdW[17], W[17];
    g.window(P + L::PRD * nS, rdW);
    double wpS[9], R[9], v4[9], dvb[9], vc[9], cvb[9];
    {
      g.window(P + L::PP * nS, W);
      const double f = rdW[8] / W[8];
#pragma unroll
      for (int o = 0; o < 9; ++o) {
        wpS[o] = f * brow<FIXED>(m, W, o);   // rho D (B p) / p of output cell j_o at s
        R[o] = bcol<FIXED>(m, rdW, o);
        cvb[o] = g.at(C + CF_VCB * nI, o) * rdW[12 - o];   // Vcbar rho D at j_o
        v4[o] = g.at(V + 4 * nI, o);
        dvb[o] = g.at(C + CF_DIVVCB * nI, o);
        vc[o] = g.at(C + CF_VC * nI, o);
      }
    }
    const double rds = rdW[8];
    const bool self = g.valid(4);
    const double divVc_s = self ? C[CF_DIVVC * nI + g.j(4)] : 0.0;
    const double Dpp_s = self ? C[CF_DPP * nI + g.j(4)] : 0.0;
#pragma unroll 1
    for (int k = 0; k < NS; ++k) {
      const double iLe = m->invLe[k], c1 = iLe * idx2;
      double hW[17], vbk[9];
      g.window(P + (L::PH + k) * nS, hW);
      const double hs = hW[8];
#pragma unroll
      for (int o = 0; o < 9; ++o) vbk[o] = g.at(V + (5 + k) * nI, o);
      const double Ys = P[(L::PY + k) * nS + s], ds = P[(L::PX + k) * nS + s] - Ys;
      double Xb = 0.0, Yb = 0.0, hb = 0.0;
      g.window(P + (L::PX + k) * nS, W);
#pragma unroll
      for (int o = 0; o < 9; ++o) hb += v4[o] * c1 * rds * brow<FIXED>(m, W, o);
#pragma unroll
      for (int mm = 0; mm < 17; ++mm) W[mm] = rdW[mm] * hW[mm];
#pragma unroll
      for (int o = 0; o < 9; ++o) {
        const double Lhb = v4[o] * c1, Lxb = (vbk[o] - dvb[o]) * c1, e = Lxb + Lhb * hs;
        const double cv = cvb[o] * iLe;
        Xb += -cv * dw[o] + e * wpS[o] + Lxb * R[o] + Lhb * bcol<FIXED>(m, W, o);
        Yb += vc[o] * dw[o] * (vbk[o] + v4[o] * hs) - e * wpS[o];
        hb += v4[o] * vc[o] * dw[o] * Ys + Lhb * ds * wpS[o];
      }
      if (self) {
        const double cv4 = cvb[4] * iLe;
        Xb -= cv4 * Dpp_s;
        Yb += (vbk[4] + v4[4] * hs) * divVc_s + cv4 * Dpp_s;
        hb += v4[4] * Ys * divVc_s;
      }
      Pb[(L::PX + k) * nS + s] += Xb;
      Pb[(L::PY + k) * nS + s] += Yb;
      Pb[(L::PH + k) * nS + s] += hb;
    }
  }
}

template <int NS, int D, bool FIXED>
__global__ __launch_bounds__(256) void k_adj_g3(const BoxDev *__restrict__ boxes,
                                                const Item *__restrict__ items, int nitems, TileShape ts,
                                                const double *__restrict__ Pbase,
                                                const double *__restrict__ Vbase,
                                                const double *__restrict__ coef, AdjBufs ab,
                                                const DevMech *__restrict__ m) {
  using L = Layout<NS>;
  constexpr int NU = L::NU, NP = L::NP;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int x, y, z;
    tile_cell(w, ts, x, y, z);
    const Gather<D> g(b, x, y, z);
    if (!g.ok) continue;
    const long long nS = g.nS, nI = g.nI;
    const int s = g.s;
    const double *P = Pbase + b.offS * NP;
    const double *V = Vbase + b.offI * NU;
    const double *C = coef + b.offI * CF_N;
    double *Pb = ab.Pb + b.offS * NP;
    const double idx = b.idx[D], idx2 = b.idx2[D];
    double dw[9];
    d1w(idx, dw);
    double rpW[17], W[17];   // rho D / p window, scratch window
    double BP[9], v4[9], dvb[9];
    double rds, ips;
    {
      double pW[17];
      g.window(P + L::PP * nS, pW);
      g.window(P + L::PRD * nS, W);
      rds = W[8];
      ips = 1.0 / pW[8];
#pragma unroll
      for (int mm = 0; mm < 17; ++mm) rpW[mm] = W[mm] / pW[mm];
#pragma unroll
      for (int o = 0; o < 9; ++o) {
        BP[o] = brow<FIXED>(m, pW, o);   // (B p)_o of output cell j_o
        v4[o] = g.at(V + 4 * nI, o);
        dvb[o] = g.at(C + CF_DIVVCB * nI, o);
      }
    }
    double wpb[9];
#pragma unroll
    for (int o = 0; o < 9; ++o) wpb[o] = 0.0;
    double rdb = 0.0, pb = 0.0;
#pragma unroll 1
    for (int k = 0; k < NS; ++k) {
      const double iLe = m->invLe[k], c1 = iLe * idx2;
      double hW[17], vbk[9];
      g.window(P + (L::PH + k) * nS, hW);
      const double hs = hW[8];
#pragma unroll
      for (int o = 0; o < 9; ++o) vbk[o] = g.at(V + (5 + k) * nI, o);
      // (B X_k) rows
      g.window(P + (L::PX + k) * nS, W);
#pragma unroll
      for (int o = 0; o < 9; ++o) rdb += brow<FIXED>(m, W, o) * ((vbk[o] - dvb[o]) * c1 + v4[o] * c1 * hs);
      // d = X_k - Y_k, then d rho D / p and h_k d rho D / p
      {
        double YW[17];
        g.window(P + (L::PY + k) * nS, YW);
#pragma unroll
        for (int mm = 0; mm < 17; ++mm) W[mm] -= YW[mm];
      }
      const double ds = W[8];
#pragma unroll
      for (int mm = 0; mm < 17; ++mm) {
        W[mm] *= rpW[mm];
        hW[mm] *= W[mm];
      }
#pragma unroll
      for (int o = 0; o < 9; ++o) {
        const double Lhb = v4[o] * c1, Lxb = (vbk[o] - dvb[o]) * c1;
        wpb[o] += (Lxb + Lhb * hs) * ds;
        pb += Lxb * bcol<FIXED>(m, W, o) + Lhb * bcol<FIXED>(m, hW, o);
      }
    }
    // rho D (B p) / p and D p / p of the output cells (p at j_o = rho D / (rho D / p))
#pragma unroll
    for (int o = 0; o < 9; ++o) {
      const double wpS = rds * BP[o] * ips;
      rdb += wpb[o] * BP[o] * ips;
      const double pj = P[L::PP * nS + min(max(s + (4 - o) * g.st, g.lo), g.hi)];
      pb += g.at(C + CF_DPPB * nI, o) * dw[o] / pj - wpb[o] * wpS * ips;
    }
    if (g.valid(4)) {
      rdb += C[CF_RDSELF * nI + g.j(4)];
      pb -= C[CF_DPPB * nI + g.j(4)] * C[CF_DPP * nI + g.j(4)] * ips;
    }
    Pb[L::PRD * nS + s] += rdb;
    Pb[L::PP * nS + s] += pb;
  }
}

// Transpose of the chemistry source rho omega_k = W_k sum_j nu_kj q_j at the
// interior cells: adds d<vbar, rho omega>/dT and /dY_k to the primitive
// adjoints, /drho to the state adjoint, and writes the workgroup's partial
// sums of d<vbar, rho omega>/d ln A_j = qbar_j q_j to partial[block][j].
// The block size must be a multiple of 64; lanes without a cell carry a zero
// cotangent through the loop so every wave reduction sees full waves.
template <int NS>
__global__ __launch_bounds__(256) void k_chem_adj(const BoxDev *__restrict__ boxes,
                                                  const Item *__restrict__ items, int nitems,
                                                  TileShape ts, const double *__restrict__ Ubase,
                                                  const double *__restrict__ Vbase, AdjBufs ab,
                                                  double *__restrict__ partial,
                                                  const DevMech *__restrict__ m, int *err) {
  using L = Layout<NS>;
  constexpr int NU = L::NU, NP = L::NP;
  __shared__ double wacc[4][NSDC_NRMAX];
  const int nr = m->nr;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int j = threadIdx.x; j < 4 * NSDC_NRMAX; j += blockDim.x) (&wacc[0][0])[j] = 0.0;
  __syncthreads();
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int x, y, z;
    tile_cell(w, ts, x, y, z);
    const bool act = x < b.nx && y < b.ny && z < b.nz;
    x = min(x, b.nx - 1);
    y = min(y, b.ny - 1);
    z = min(z, b.nz - 1);
    const long long nS = (long long)b.sx * b.sy * b.sz, nI = (long long)b.nx * b.ny * b.nz;
    const long long s = ((long long)(z + NSDC_NG) * b.sy + (y + NSDC_NG)) * b.sx + (x + NSDC_NG);
    const long long i = ((long long)z * b.ny + y) * b.nx + x;
    const double *U = Ubase + b.offS * NU;
    const double *V = Vbase + b.offI * NU;
    double Uc[NU];
#pragma unroll
    for (int q = 0; q < NU; ++q) Uc[q] = U[q * nS + s];
    double rho, u[3], Y[NS], T;
    const int e = cell_state<NS>(m, Uc, rho, u, Y, T);
    if (e && act) atomicOr(err, e);
    const double lnT = log(T), invT = 1.0 / T;
    const double lnRTp = lnT + LN_RU_PREF;
    double c[NS + 1], g[NS + 1], hr[NS + 1], wb[NS + 1], cb[NS + 1];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      c[k] = rho * Y[k] * m->invW[k];
      hr[k] = h_RT(m, k, T, invT);
      g[k] = hr[k] - s_R(m, k, T, lnT);
      wb[k] = act ? V[(5 + k) * nI + i] * m->W[k] : 0.0;
      cb[k] = 0.0;
    }
    c[NS] = 1.0;
    g[NS] = hr[NS] = wb[NS] = cb[NS] = 0.0;
    double Tb = 0.0;
#pragma unroll 2
    for (int j = 0; j < nr; ++j) {
      const int r0 = m->rs[j][0], r1 = m->rs[j][1], p0 = m->ps[j][0], p1 = m->ps[j][1];
      const double dlnkf = m->beta[j] * invT + m->EaR[j] * invT * invT;
      const double lnkf = m->lnA[j] + m->beta[j] * lnT - m->EaR[j] * invT;
      const double dg = (g[p0] + g[p1]) - (g[r0] + g[r1]);
      const double dh = (hr[p0] + hr[p1]) - (hr[r0] + hr[r1]);
      const double kf = exp(lnkf);
      const double kr = exp(lnkf + dg + m->dnu[j] * lnRTp);
      const double fw = kf * c[r0] * c[r1], rv = kr * c[p0] * c[p1];
      const double qb = (wb[p0] + wb[p1]) - (wb[r0] + wb[r1]);
      cb[r0] += qb * kf * c[r1];
      cb[r1] += qb * kf * c[r0];
      cb[p0] -= qb * kr * c[p1];
      cb[p1] -= qb * kr * c[p0];
      // d ln k_r / dT = d ln k_f / dT - sum nu h/(R T^2) + dnu / T
      Tb += qb * (fw * dlnkf - rv * (dlnkf + (m->dnu[j] - dh) * invT));
      const double sum = wave_sum(qb * (fw - rv));
      if (lane == 0) wacc[wave][j] += sum;
    }
    if (!act) continue;
    double *Pb = ab.Pb + b.offS * NP;
    double rhob = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      rhob += cb[k] * Y[k] * m->invW[k];
      Pb[(L::PY + k) * nS + s] += cb[k] * rho * m->invW[k];
    }
    Pb[L::PT * nS + s] += Tb;
    ab.Ub[b.offS * NU + s] += rhob;
  }
  __syncthreads();
  const int nw = (blockDim.x + 63) >> 6;
  for (int j = threadIdx.x; j < nr; j += blockDim.x) {
    double sum = 0.0;
    for (int q = 0; q < nw; ++q) sum += wacc[q][j];
    partial[(long long)blockIdx.x * nr + j] = sum;
  }
}

// Transpose of G[3 j + i] = D_j u_i: ubar_i(s) += (1/dx_j) sum_m C_m
// (Gbar(s - m e_j) - Gbar(s + m e_j)) over the cells where G was formed
// (interior j-coordinate).
template <int NS>
__global__ __launch_bounds__(256) void k_vgrad_adj(const BoxDev *__restrict__ boxes,
                                                   const Item *__restrict__ items, int nitems,
                                                   TileShape ts, AdjBufs ab) {
  using L = Layout<NS>;
  const double Cm[4] = {C1, C2, C3, C4};
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int x, y, z;
    tile_cell(w, ts, x, y, z);
    if (x >= b.sx || y >= b.sy || z >= b.sz) continue;
    const long long nS = (long long)b.sx * b.sy * b.sz;
    const long long s = ((long long)z * b.sy + y) * b.sx + x;
    const double *Gb = ab.Gb + b.offS * 9;
    double *Pb = ab.Pb + b.offS * L::NP;
    const int c[3] = {x, y, z};
    const int n[3] = {b.nx, b.ny, b.nz};
    const long long st[3] = {1, b.sx, (long long)b.sx * b.sy};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double a = 0.0;
#pragma unroll
        for (int mm = 1; mm <= 4; ++mm) {
          if (c[j] - mm >= NSDC_NG && c[j] - mm < n[j] + NSDC_NG) a += Cm[mm - 1] * Gb[(3 * j + i) * nS + s - mm * st[j]];
          if (c[j] + mm >= NSDC_NG && c[j] + mm < n[j] + NSDC_NG) a -= Cm[mm - 1] * Gb[(3 * j + i) * nS + s + mm * st[j]];
        }
        acc += a * b.idx[j];
      }
      Pb[(L::PU + i) * nS + s] += acc;
    }
  }
}

// Transpose of the conserved -> primitive map at every stored cell:
// Ub(s) += (d prim / dU)^T Pb(s), in place.
template <int NS>
__global__ __launch_bounds__(256) void k_prims_adj(const BoxDev *__restrict__ boxes,
                                                   const Item *__restrict__ items, int nitems,
                                                   TileShape ts, const double *__restrict__ Ubase,
                                                   AdjBufs ab, const DevMech *__restrict__ m, int *err) {
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
    const double *U = Ubase + b.offS * NU;
    const double *Pb = ab.Pb + b.offS * NP;
    double *Ub = ab.Ub + b.offS * NU;
    double Uc[NU];
#pragma unroll
    for (int q = 0; q < NU; ++q) Uc[q] = U[q * nS + s];
    double rho, u[3], Y[NS], T;
    const int e = cell_state<NS>(m, Uc, rho, u, Y, T);
    if (e) atomicOr(err, e);
    const double invT = 1.0 / T, ir = 1.0 / rho;
    double sumYW = 0.0, cp = 0.0, dcp = 0.0, cv = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const double *a = m->cp[k];
      const double cpk = cp_R(m, k, T);
      sumYW += Y[k] * m->invW[k];
      cp += Y[k] * m->Rk[k] * cpk;
      dcp += Y[k] * m->Rk[k] * (a[1] + T * (2.0 * a[2] + T * (3.0 * a[3] + T * 4.0 * a[4])));
      cv += Y[k] * m->Rk[k] * (cpk - 1.0);
    }
    const double Wbar = 1.0 / sumYW;
    const double mu = m->mu_ref * pow(T * m->inv_Tref, m->mu_exp);
    double ubar[3], Yb[NS];
#pragma unroll
    for (int d = 0; d < 3; ++d) ubar[d] = Pb[(L::PU + d) * nS + s];
    double Tb = Pb[L::PT * nS + s];
    const double pbar = Pb[L::PP * nS + s];
    const double lamb = Pb[L::PLAM * nS + s];
    // rho D = lambda / c_p = mu / Pr; lambda = mu c_p / Pr
    const double mub = Pb[L::PMU * nS + s] + (lamb * cp + Pb[L::PRD * nS + s]) * m->inv_Pr;
    const double cpb = lamb * mu * m->inv_Pr;
    Tb += mub * m->mu_exp * mu * invT + cpb * dcp + pbar * rho * RU * sumYW;
    double XX = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) XX += Pb[(L::PX + k) * nS + s] * Y[k] * m->invW[k] * Wbar;
    double rhob = pbar * RU * T * sumYW;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      Tb += Pb[(L::PH + k) * nS + s] * m->Rk[k] * cp_R(m, k, T);
      Yb[k] = Pb[(L::PY + k) * nS + s] + cpb * m->Rk[k] * cp_R(m, k, T) +
              m->invW[k] * Wbar * (Pb[(L::PX + k) * nS + s] - XX) + pbar * rho * RU * T * m->invW[k];
    }
    // T(e, Y): dT = (de - sum_k e_k dY_k) / c_v
    const double eb = Tb / cv;
#pragma unroll
    for (int k = 0; k < NS; ++k) Yb[k] -= eb * m->Rk[k] * T * (h_RT(m, k, T, invT) - 1.0);
    // e = U_4 / rho - |u|^2 / 2, u = U_{1..3} / rho, Y = U_{5+k} / rho
    Ub[4 * nS + s] += eb * ir;
    rhob -= eb * Uc[4] * ir * ir;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double ud = ubar[d] - eb * u[d];
      Ub[(1 + d) * nS + s] += ud * ir;
      rhob -= ud * u[d] * ir;
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      Ub[(5 + k) * nS + s] += Yb[k] * ir;
      rhob -= Yb[k] * Y[k] * ir;
    }
    Ub[s] += rhob;
  }
}

// Interior adjoint += sum of the stored-cell adjoints over the periodic
// images of each interior cell.
template <int NU>
__global__ __launch_bounds__(256) void k_fold(const BoxDev *__restrict__ boxes,
                                              const Item *__restrict__ items, int nitems,
                                              TileShape ts, AdjBufs ab, double *__restrict__ out) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int x, y, z;
    tile_cell(w, ts, x, y, z);
    if (x >= b.nx || y >= b.ny || z >= b.nz) continue;
    const long long nS = (long long)b.sx * b.sy * b.sz, nI = (long long)b.nx * b.ny * b.nz;
    const long long i = ((long long)z * b.ny + y) * b.nx + x;
    const double *Ub = ab.Ub + b.offS * NU;
    double *O = out + b.offI * NU;
    // stored coordinates congruent to the cell: c + NG + k n within [0, n + 8)
    const int c[3] = {x, y, z}, n[3] = {b.nx, b.ny, b.nz};
    int lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = c[d] + NSDC_NG;
      while (lo[d] - n[d] >= 0) lo[d] -= n[d];
      hi[d] = lo[d];
      while (hi[d] + n[d] < n[d] + 2 * NSDC_NG) hi[d] += n[d];
    }
    for (int q = 0; q < NU; ++q) {
      double sum = 0.0;
      for (int zs = lo[2]; zs <= hi[2]; zs += n[2])
        for (int ys = lo[1]; ys <= hi[1]; ys += n[1])
          for (int xs = lo[0]; xs <= hi[0]; xs += n[0])
            sum += Ub[q * nS + ((long long)zs * b.sy + ys) * b.sx + xs];
      O[q * nI + i] += sum;
    }
  }
}

// lnA_bar[j] += sum over workgroups of partial[block][j]: workgroup j sums
// reaction j's partials, thread t taking blocks t, t + 256, ... in order,
// then a fixed binary tree over the threads (deterministic).
__global__ __launch_bounds__(256) void k_lnA_reduce(const double *__restrict__ partial, int nblocks,
                                                    int nr, double *__restrict__ lnA_bar) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int q = threadIdx.x; q < nblocks; q += 256) s += partial[(long long)q * nr + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) lnA_bar[j] += red[0];
}

// ------------------------------------------------------------------ launches
static inline int grid_of(int nitems, int cap) { return nitems < cap ? (nitems > 0 ? nitems : 1) : cap; }
static inline int flat_grid(long long n) {
  const long long g = (n + 255) / 256;
  return (int)(g < 8192 ? (g > 0 ? g : 1) : 8192);
}

template <int NS>
struct AdjLaunch {
  template <int D, bool FIXED>
  static void dir_dt(const LaunchCtx &c, const double *U, const double *P, const double *G, const double *V,
                     const AdjBufs &ab, double *coef, unsigned parts) {
    const dim3 gI(grid_of(c.nI, c.cap)), bI(c.tsI.tx * c.tsI.ty * c.tsI.tz);
    const dim3 gS(grid_of(c.nS, c.cap)), bS(c.tsS.tx * c.tsS.ty * c.tsS.tz);
    prof_begin(c.prof, K_DIR_ADJ_X + D, c.stream);
    if (parts & 2)
      hipLaunchKernelGGL((k_adj_coef<NS, D, FIXED>), gI, bI, 0, c.stream, c.boxes, c.itemsI, c.nI, c.tsI, P, V,
                         coef, c.mech);
    hipLaunchKernelGGL((k_adj_g1<NS, D, FIXED>), gS, bS, 0, c.stream, c.boxes, c.itemsS, c.nS, c.tsS, U, P, G, V,
                       ab, parts, c.mech);
    if (parts & 2) {
      hipLaunchKernelGGL((k_adj_g2<NS, D, FIXED>), gS, bS, 0, c.stream, c.boxes, c.itemsS, c.nS, c.tsS, P, V,
                         coef, ab, c.mech);
      hipLaunchKernelGGL((k_adj_g3<NS, D, FIXED>), gS, bS, 0, c.stream, c.boxes, c.itemsS, c.nS, c.tsS, P, V,
                         coef, ab, c.mech);
    }
    prof_end(c.prof, K_DIR_ADJ_X + D, c.stream);
  }
  template <bool FIXED>
  static void dir_t(const LaunchCtx &c, int d, const double *U, const double *P, const double *G,
                    const double *V, const AdjBufs &ab, double *coef, unsigned parts) {
    if (d == 0)
      dir_dt<0, FIXED>(c, U, P, G, V, ab, coef, parts);
    else if (d == 1)
      dir_dt<1, FIXED>(c, U, P, G, V, ab, coef, parts);
    else
      dir_dt<2, FIXED>(c, U, P, G, V, ab, coef, parts);
  }
  static void dir(const LaunchCtx &c, int d, const double *U, const double *P, const double *G,
                  const double *V, const AdjBufs &ab, double *coef, unsigned parts) {
    if (c.smc_stencil)
      dir_t<true>(c, d, U, P, G, V, ab, coef, parts);
    else
      dir_t<false>(c, d, U, P, G, V, ab, coef, parts);
  }
  static int chem(const LaunchCtx &c, const double *U, const double *V, const AdjBufs &ab, double *partial) {
    const int grid = grid_of(c.nI, c.cap);
    prof_begin(c.prof, K_CHEM_ADJ, c.stream);
    hipLaunchKernelGGL(k_chem_adj<NS>, dim3(grid), dim3(c.tsI.tx * c.tsI.ty * c.tsI.tz), 0, c.stream, c.boxes,
                       c.itemsI, c.nI, c.tsI, U, V, ab, partial, c.mech, c.err);
    prof_end(c.prof, K_CHEM_ADJ, c.stream);
    return grid;
  }
  static void vgrad(const LaunchCtx &c, const AdjBufs &ab) {
    prof_begin(c.prof, K_VGRAD_ADJ, c.stream);
    hipLaunchKernelGGL(k_vgrad_adj<NS>, dim3(grid_of(c.nS, c.cap)), dim3(c.tsS.tx * c.tsS.ty * c.tsS.tz), 0,
                       c.stream, c.boxes, c.itemsS, c.nS, c.tsS, ab);
    prof_end(c.prof, K_VGRAD_ADJ, c.stream);
  }
  static void prims(const LaunchCtx &c, const double *U, const AdjBufs &ab) {
    prof_begin(c.prof, K_PRIMS_ADJ, c.stream);
    hipLaunchKernelGGL(k_prims_adj<NS>, dim3(grid_of(c.nS, c.cap)), dim3(c.tsS.tx * c.tsS.ty * c.tsS.tz), 0,
                       c.stream, c.boxes, c.itemsS, c.nS, c.tsS, U, ab, c.mech, c.err);
    prof_end(c.prof, K_PRIMS_ADJ, c.stream);
  }
  static void fold(const LaunchCtx &c, const AdjBufs &ab, double *out) {
    prof_begin(c.prof, K_FOLD, c.stream);
    hipLaunchKernelGGL(k_fold<5 + NS>, dim3(grid_of(c.nI, c.cap)), dim3(c.tsI.tx * c.tsI.ty * c.tsI.tz), 0,
                       c.stream, c.boxes, c.itemsI, c.nI, c.tsI, ab, out);
    prof_end(c.prof, K_FOLD, c.stream);
  }
};

void adj_fill0(const LaunchCtx &c, double *p, long long n) {
  prof_begin(c.prof, K_ADJ_LINALG, c.stream);
  hipLaunchKernelGGL(k_fill0, dim3(flat_grid(n)), dim3(256), 0, c.stream, p, n);
  prof_end(c.prof, K_ADJ_LINALG, c.stream);
}
void adj_axpy(const LaunchCtx &c, const double *X, const AxpyArgs &a, long long n) {
  prof_begin(c.prof, K_ADJ_LINALG, c.stream);
  hipLaunchKernelGGL(k_axpy_multi, dim3(flat_grid(n)), dim3(256), 0, c.stream, X, a, n);
  prof_end(c.prof, K_ADJ_LINALG, c.stream);
}
void adj_lincomb(const LaunchCtx &c, const LincombArgs &a, double *Y, long long n) {
  prof_begin(c.prof, K_ADJ_LINALG, c.stream);
  hipLaunchKernelGGL(k_lincomb, dim3(flat_grid(n)), dim3(256), 0, c.stream, a, Y, n);
  prof_end(c.prof, K_ADJ_LINALG, c.stream);
}
void adj_lnA_reduce(const LaunchCtx &c, const double *partial, int nblocks, int nr, double *lnA_bar) {
  prof_begin(c.prof, K_ADJ_LINALG, c.stream);
  hipLaunchKernelGGL(k_lnA_reduce, dim3(nr), dim3(256), 0, c.stream, partial, nblocks, nr, lnA_bar);
  prof_end(c.prof, K_ADJ_LINALG, c.stream);
}

template <int NS>
static const AdjOps make_adj_ops() {
  AdjOps o;
  o.ns = NS;
  o.dir = &AdjLaunch<NS>::dir;
  o.chem = &AdjLaunch<NS>::chem;
  o.vgrad = &AdjLaunch<NS>::vgrad;
  o.prims = &AdjLaunch<NS>::prims;
  o.fold = &AdjLaunch<NS>::fold;
  return o;
}
#define NSDC_ADJ_DEF(n) static const AdjOps ADJ_##n = make_adj_ops<n>();
NSDC_SPECIES_COUNTS(NSDC_ADJ_DEF)
#undef NSDC_ADJ_DEF

const AdjOps *adj_ops_for(int ns) {
#define NSDC_ADJ_CASE(n) \
  if (ns == (n)) return &ADJ_##n;
  NSDC_SPECIES_COUNTS(NSDC_ADJ_CASE)
#undef NSDC_ADJ_CASE
  return nullptr;
}

}  // namespace nsdc
