// Device kernels of the vector-Jacobian product of the right-hand side (the
// adjoint of eq. cns as discretised in Section 2.2), FP64, gfx950.
//
// Given a cotangent vbar of dU/dt on the interior, the product
// Ubar = (d rhs / dU)^T vbar is formed stage by stage in reverse:
//   k_dir_adj<D>   transpose of every term that differentiates along D.  A
//                  thread takes one output cell, re-forms the forward
//                  quantities of its nine-point line and adds the partial
//                  derivatives of <vbar, rhs> to the adjoints of the sampled
//                  primitive, state and velocity-gradient fields.  Output
//                  cells nine apart along D touch disjoint lines, so the
//                  cells with c_D = 9 t + r (phase r) are one launch with
//                  plain read-add-write updates: nine launches per direction,
//                  in a fixed order, no atomics.
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

template <int NS, int D, bool FIXED>
__global__ __launch_bounds__(256) void k_dir_adj(const BoxDev *__restrict__ boxes,
                                                 const Item *__restrict__ items, int nitems,
                                                 TileShape ts, int phase,
                                                 const double *__restrict__ Ubase,
                                                 const double *__restrict__ Pbase,
                                                 const double *__restrict__ Gbase,
                                                 const double *__restrict__ Vbase, AdjBufs ab,
                                                 unsigned parts, const DevMech *__restrict__ m) {
  using L = Layout<NS>;
  constexpr int NU = L::NU, NP = L::NP;
  constexpr int J1 = D == 0 ? 1 : 0, J2 = D == 2 ? 1 : 2;   // the two other directions
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int c[3];
    tile_cell(w, ts, c[0], c[1], c[2]);
    c[D] = 9 * c[D] + phase;
    if (c[0] >= b.nx || c[1] >= b.ny || c[2] >= b.nz) continue;
    const long long nS = (long long)b.sx * b.sy * b.sz;
    const long long nI = (long long)b.nx * b.ny * b.nz;
    const long long s = ((long long)(c[2] + NSDC_NG) * b.sy + (c[1] + NSDC_NG)) * b.sx + (c[0] + NSDC_NG);
    const long long i = ((long long)c[2] * b.ny + c[1]) * b.nx + c[0];
    const long long st = D == 0 ? 1 : (D == 1 ? (long long)b.sx : (long long)b.sx * b.sy);
    const double *U = Ubase + b.offS * NU;
    const double *P = Pbase + b.offS * NP;
    const double *G = Gbase + b.offS * 9;
    const double *V = Vbase + b.offI * NU;
    double *Ub = ab.Ub + b.offS * NU;
    double *Pb = ab.Pb + b.offS * NP;
    double *Gb = ab.Gb + b.offS * 9;
    const double idx = b.idx[D], idx2 = b.idx2[D];
    auto line = [&](const double *f, double *v) {
#pragma unroll
      for (int o = 0; o < 9; ++o) v[o] = f[s + (o - 4) * st];
    };
    auto scat = [&](double *f, const double *v) {
#pragma unroll
      for (int o = 0; o < 9; ++o) f[s + (o - 4) * st] += v[o];
    };
    double vb[NU];
#pragma unroll
    for (int q = 0; q < NU; ++q) vb[q] = V[q * nI + i];
    double dw[9];
    d1w(idx, dw);
    double uu[3][9], pp[9];
#pragma unroll
    for (int ic = 0; ic < 3; ++ic) line(P + (L::PU + ic) * nS, uu[ic]);
    line(P + L::PP * nS, pp);
    // adjoints of the velocity and pressure samples, scattered at the end
    double ub[3][9], pb[9];
#pragma unroll
    for (int o = 0; o < 9; ++o) {
      ub[0][o] = ub[1][o] = ub[2][o] = 0.0;
      pb[o] = 0.0;
    }

    if (parts & 1) {  // -D_D(F_D(U))
      double f[9], t[9];
#pragma unroll
      for (int o = 0; o < 9; ++o) t[o] = -vb[0] * dw[o];
      scat(Ub + (1 + D) * nS, t);
#pragma unroll
      for (int ic = 0; ic < 3; ++ic) {
        line(U + (1 + ic) * nS, f);
        const double a = -vb[1 + ic];
#pragma unroll
        for (int o = 0; o < 9; ++o) {
          const double ao = a * dw[o];
          t[o] = ao * uu[D][o];
          ub[D][o] += ao * f[o];
          if (ic == D) pb[o] += ao;
        }
        scat(Ub + (1 + ic) * nS, t);
      }
      line(U + 4 * nS, f);
#pragma unroll
      for (int o = 0; o < 9; ++o) {
        const double ao = -vb[4] * dw[o];
        t[o] = ao * uu[D][o];
        pb[o] += ao * uu[D][o];
        ub[D][o] += ao * (f[o] + pp[o]);
      }
      scat(Ub + 4 * nS, t);
#pragma unroll 1
      for (int k = 0; k < NS; ++k) {
        line(U + (5 + k) * nS, f);
        const double a = -vb[5 + k];
#pragma unroll
        for (int o = 0; o < 9; ++o) {
          const double ao = a * dw[o];
          t[o] = ao * uu[D][o];
          ub[D][o] += ao * f[o];
        }
        scat(Ub + (5 + k) * nS, t);
      }
    }

    if (parts & 2) {
      const double bulk = m->bulk;
      const double lam2 = bulk - 2.0 / 3.0;
      const double ewD = 1.0 / 3.0 + bulk;
      double mu[9], mub[9], v[9], bt[9], t[9];
      line(P + L::PMU * nS, mu);
      // every L_D(mu, .) term at once: sum_ic vb_ic c_ic L(mu, u_ic) +
      // vb_E [(1/3 + xi) L(mu, u_D^2/2) + L(mu, |u|^2/2)]
#pragma unroll
      for (int o = 0; o < 9; ++o) {
        double phi = vb[4] * (ewD * 0.5 * uu[D][o] * uu[D][o] +
                              0.5 * (uu[0][o] * uu[0][o] + uu[1][o] * uu[1][o] + uu[2][o] * uu[2][o]));
#pragma unroll
        for (int ic = 0; ic < 3; ++ic) phi += vb[1 + ic] * (ic == D ? 4.0 / 3.0 + bulk : 1.0) * uu[ic][o];
        t[o] = phi;
      }
      bvec<FIXED>(m, t, v);
#pragma unroll
      for (int o = 0; o < 9; ++o) mub[o] = idx2 * v[o];
      btvec<FIXED>(m, mu, bt);
#pragma unroll
      for (int ic = 0; ic < 3; ++ic) {
        const double cic = vb[1 + ic] * (ic == D ? 4.0 / 3.0 + bulk : 1.0);
        const double ce = vb[4] * (ic == D ? 1.0 + ewD : 1.0);
#pragma unroll
        for (int o = 0; o < 9; ++o) ub[ic][o] += idx2 * bt[o] * (cic + ce * uu[ic][o]);
      }
      // D_D((xi - 2/3 mu) sum_{j != D} D_j u_j) and its viscous work
      {
        double g1[9], g2[9];
        line(G + (3 * J1 + J1) * nS, g1);
        line(G + (3 * J2 + J2) * nS, g2);
#pragma unroll
        for (int o = 0; o < 9; ++o) {
          const double gs = g1[o] + g2[o];
          const double gbar = dw[o] * (vb[1 + D] + vb[4] * uu[D][o]);
          ub[D][o] += vb[4] * dw[o] * lam2 * mu[o] * gs;
          mub[o] += gbar * lam2 * gs;
          t[o] = gbar * lam2 * mu[o];
        }
        scat(Gb + (3 * J1 + J1) * nS, t);
        scat(Gb + (3 * J2 + J2) * nS, t);
      }
      // D_D(mu D_ic u_D), ic != D, and its viscous work
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int ic = e == 0 ? J1 : J2;
        double gg[9];
        line(G + (3 * ic + D) * nS, gg);
#pragma unroll
        for (int o = 0; o < 9; ++o) {
          const double gbar = dw[o] * (vb[1 + ic] + vb[4] * uu[ic][o]);
          ub[ic][o] += vb[4] * dw[o] * mu[o] * gg[o];
          mub[o] += gbar * gg[o];
          t[o] = gbar * mu[o];
        }
        scat(Gb + (3 * ic + D) * nS, t);
      }
      scat(Pb + L::PMU * nS, mub);
      // heat conduction L_D(lambda, T)
      {
        double T9[9], lam[9];
        line(P + L::PT * nS, T9);
        line(P + L::PLAM * nS, lam);
        bvec<FIXED>(m, T9, v);
#pragma unroll
        for (int o = 0; o < 9; ++o) t[o] = vb[4] * idx2 * v[o];
        scat(Pb + L::PLAM * nS, t);
        btvec<FIXED>(m, lam, bt);
#pragma unroll
        for (int o = 0; o < 9; ++o) t[o] = vb[4] * idx2 * bt[o];
        scat(Pb + L::PT * nS, t);
      }
      // species diffusion and the correction velocity
      {
        double rd[9], rdb[9], Bp[9], wp[9], wpb[9];
        line(P + L::PRD * nS, rd);
        bvec<FIXED>(m, pp, Bp);
#pragma unroll
        for (int o = 0; o < 9; ++o) {
          wp[o] = rd[o] * Bp[o] / pp[o];
          rdb[o] = 0.0;
          wpb[o] = 0.0;
        }
        const double Dpp = d1(pp, idx) / pp[4];
        const double rd4 = rd[4];
        // forward values divVc, Vc and the adjoints of both
        double divVc = 0.0, Vc = 0.0, divVcb = 0.0, Vcb = 0.0, S1 = 0.0, S2 = 0.0;
#pragma unroll 1
        for (int k = 0; k < NS; ++k) {
          const double iLe = m->invLe[k];
          double X9[9], Y9[9], h9[9];
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
          divVcb += (vb[5 + k] + vb[4] * h9[4]) * Y9[4];
          Vcb += vb[5 + k] * d1(Y9, idx) + vb[4] * d1p(h9, Y9, idx);
        }
        rdb[4] -= Vcb * S1;
        const double Dppb = -Vcb * rd4 * S2;
#pragma unroll 1
        for (int k = 0; k < NS; ++k) {
          const double iLe = m->invLe[k];
          double X9[9], Y9[9], h9[9], Xb[9], Yb[9], hb[9];
          line(P + (L::PX + k) * nS, X9);
          line(P + (L::PY + k) * nS, Y9);
          line(P + (L::PH + k) * nS, h9);
          bvec<FIXED>(m, X9, v);
          const double Lxb = (vb[5 + k] - divVcb) * iLe * idx2;
          const double Lhb = vb[4] * iLe * idx2;
          const double cv = Vcb * rd4 * iLe;
#pragma unroll
          for (int o = 0; o < 9; ++o) {
            const double e = Lxb + Lhb * h9[o];
            const double d = X9[o] - Y9[o];
            const double db = e * wp[o];
            t[o] = rd[o] * e;
            Xb[o] = -cv * dw[o] + db;
            Yb[o] = Vc * dw[o] * (vb[5 + k] + vb[4] * h9[o]) - db;
            hb[o] = vb[4] * Vc * dw[o] * Y9[o] + Lhb * (rd[o] * v[o] + d * wp[o]);
            rdb[o] += v[o] * e;
            wpb[o] += e * d;
          }
          Xb[4] -= cv * Dpp;
          Yb[4] += (vb[5 + k] + vb[4] * h9[4]) * divVc + cv * Dpp;
          hb[4] += vb[4] * Y9[4] * divVc;
          btvec<FIXED>(m, t, bt);
#pragma unroll
          for (int o = 0; o < 9; ++o) Xb[o] += bt[o];
          scat(Pb + (L::PX + k) * nS, Xb);
          scat(Pb + (L::PY + k) * nS, Yb);
          scat(Pb + (L::PH + k) * nS, hb);
        }
        // wp = rd (B p) / p and Dpp = D p / p_centre
#pragma unroll
        for (int o = 0; o < 9; ++o) {
          rdb[o] += wpb[o] * Bp[o] / pp[o];
          t[o] = wpb[o] * rd[o] / pp[o];
          pb[o] += Dppb * dw[o] / pp[4] - wpb[o] * wp[o] / pp[o];
        }
        pb[4] -= Dppb * Dpp / pp[4];
        btvec<FIXED>(m, t, bt);
#pragma unroll
        for (int o = 0; o < 9; ++o) pb[o] += bt[o];
        scat(Pb + L::PRD * nS, rdb);
      }
    }
#pragma unroll
    for (int ic = 0; ic < 3; ++ic) scat(Pb + (L::PU + ic) * nS, ub[ic]);
    scat(Pb + L::PP * nS, pb);
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
    const double lnRTp = log(RU * T / PREF);
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

// lnA_bar[j] += sum over workgroups of partial[block][j], in block order.
__global__ __launch_bounds__(256) void k_lnA_reduce(const double *__restrict__ partial, int nblocks,
                                                    int nr, double *__restrict__ lnA_bar) {
  for (int j = threadIdx.x; j < nr; j += blockDim.x) {
    double s = 0.0;
    for (int q = 0; q < nblocks; ++q) s += partial[(long long)q * nr + j];
    lnA_bar[j] += s;
  }
}

// ------------------------------------------------------------------ launches
static inline int grid_of(int nitems, int cap) { return nitems < cap ? (nitems > 0 ? nitems : 1) : cap; }
static inline int flat_grid(long long n) {
  const long long g = (n + 255) / 256;
  return (int)(g < 8192 ? (g > 0 ? g : 1) : 8192);
}

template <int NS>
struct AdjLaunch {
  template <bool FIXED>
  static void dir_t(const LaunchCtx &c, const AdjItems &ai, int d, int phase, const double *U,
                    const double *P, const double *G, const double *V, const AdjBufs &ab, unsigned parts) {
    const dim3 grid(grid_of(ai.n[d], c.cap)), block(ai.ts[d].tx * ai.ts[d].ty * ai.ts[d].tz);
    const Item *items = ai.items[d];
    prof_begin(c.prof, K_DIR_ADJ_X + d, c.stream);
    if (d == 0)
      hipLaunchKernelGGL((k_dir_adj<NS, 0, FIXED>), grid, block, 0, c.stream, c.boxes, items, ai.n[d], ai.ts[d],
                         phase, U, P, G, V, ab, parts, c.mech);
    else if (d == 1)
      hipLaunchKernelGGL((k_dir_adj<NS, 1, FIXED>), grid, block, 0, c.stream, c.boxes, items, ai.n[d], ai.ts[d],
                         phase, U, P, G, V, ab, parts, c.mech);
    else
      hipLaunchKernelGGL((k_dir_adj<NS, 2, FIXED>), grid, block, 0, c.stream, c.boxes, items, ai.n[d], ai.ts[d],
                         phase, U, P, G, V, ab, parts, c.mech);
    prof_end(c.prof, K_DIR_ADJ_X + d, c.stream);
  }
  static void dir(const LaunchCtx &c, const AdjItems &ai, int d, int phase, const double *U, const double *P,
                  const double *G, const double *V, const AdjBufs &ab, unsigned parts) {
    if (c.smc_stencil)
      dir_t<true>(c, ai, d, phase, U, P, G, V, ab, parts);
    else
      dir_t<false>(c, ai, d, phase, U, P, G, V, ab, parts);
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
  hipLaunchKernelGGL(k_lnA_reduce, dim3(1), dim3(256), 0, c.stream, partial, nblocks, nr, lnA_bar);
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
static const AdjOps ADJ9 = make_adj_ops<9>();
static const AdjOps ADJ21 = make_adj_ops<21>();

const AdjOps *adj_ops_for(int ns) {
  switch (ns) {
    case 9: return &ADJ9;
    case 21: return &ADJ21;
    default: return nullptr;
  }
}

}  // namespace nsdc
