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

#include <type_traits>

#include "nsdc_internal.h"

#include "physics.h"

namespace nsdc {

// LDS bytes a workgroup of the chemistry kernels may take for the per-cell
// species arrays (gfx950: up to 160 KiB per workgroup)
#ifndef NSDC_CHEM_LDS_LIMIT
#define NSDC_CHEM_LDS_LIMIT 163840
#endif

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
                                               FRef Uref, const int *__restrict__ skip) {
  if (skip && *skip) return;   // a residual early exit ended the step's sweeps
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
    // the periodic image, or along a direction with physical boundaries the
    // nearest boundary cell (a finite state no stencil reads)
    auto src_of = [&](int c, int n, int d) {
      return ((b.np >> d) & 1) ? min(max(c - NSDC_NG, 0), n - 1) + NSDC_NG : ((c - NSDC_NG) % n + n) % n + NSDC_NG;
    };
    const int xs = src_of(x, b.nx, 0), ys = src_of(y, b.ny, 1), zs = src_of(z, b.nz, 2);
    const long long nS = (long long)b.sx * b.sy * b.sz;
    const long long dst = ((long long)z * b.sy + y) * b.sx + x;
    const long long src = ((long long)zs * b.sy + ys) * b.sx + xs;
    double *U = Uref.get(w.box, b.offS * NCOMP);
#pragma unroll 4
    for (int q = 0; q < NCOMP; ++q) U[q * nS + dst] = U[q * nS + src];
  }
}

// out_mode: 0 leave the right-hand side alone, 1 zero it, 2 chemistry source
// (only the CHEM instance takes mode 2: without the chemistry the kernel
// needs fewer registers, and it is held to three waves per SIMD, 168
// registers: at 21 species the compiler's 183 registers allowed two waves
// and the kernel took 12% longer).
// warm != 0: start the Newton solve from the temperature the previous
// evaluation left in P (when it lies in the fit range), else from 1000 K.
template <int NS, bool CHEM>
__global__ __launch_bounds__(256, CHEM ? 2 : 3) void k_prims(const BoxDev *__restrict__ boxes,
                                               const Item *__restrict__ items, int nitems,
                                               TileShape ts, FRef Uref, double *__restrict__ Pbase,
                                               FRef Fout, int out_mode, int warm, int store_x,
                                               const DevMech *__restrict__ m, int *err,
                                               const int *__restrict__ skip) {
  if (skip && *skip) return;   // a residual early exit ended the step's sweeps
  using L = Layout<NS>;
  constexpr int NU = L::NU, NP = L::NP;
  constexpr int LIM = CHEM ? 65536 : 0;
  NSDC_CHEM_LDS(NS, LIM, chem_sh);
  double *sh = chem_lds_setup<NS, LIM>(chem_sh, m);
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
    double T0 = 1000.0;
    if (warm) {
      const double Tp = P[L::PT * nS + s];
      if (Tp >= m->Tlo && Tp <= m->Thi) T0 = Tp;
    }
    const int e = cell_state<NS>(m, Uc, rho, u, Y, T, T0);
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
    P[L::PWB * nS + s] = Wbar;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      P[(L::PY + k) * nS + s] = Y[k];
      if (store_x) {
        P[(L::PX + k) * nS + s] = Y[k] * Wbar * m->invW[k];
        P[(L::PH + k) * nS + s] = m->Rk[k] * T * h_RT(m, k, T, invT);
      }
    }
    if (out_mode == 0) continue;
    const int xi = x - NSDC_NG, yi = y - NSDC_NG, zi = z - NSDC_NG;
    if (xi < 0 || yi < 0 || zi < 0 || xi >= b.nx || yi >= b.ny || zi >= b.nz) continue;
    const long long nI = (long long)b.nx * b.ny * b.nz;
    const long long i = ((long long)zi * b.ny + yi) * b.nx + xi;
    double *F = Fout.get(w.box, b.offI * NU);
#pragma unroll
    for (int q = 0; q < 5; ++q) F[q * nI + i] = 0.0;
    if (CHEM && out_mode == 2) {
      double wd[NS];
      production_any<NS, LIM>(m, rho, T, Y, wd, sh);
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
                                               double *__restrict__ Gbase, const DevMech *__restrict__ m,
                                               const int *__restrict__ skip) {
  if (skip && *skip) return;   // a residual early exit ended the step's sweeps
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
      // within 4 cells of a physical boundary along j: its diffusive
      // first-derivative stencil (Section 2.5)
      const int cj = c[j] - NSDC_NG, bj = min(cj, n[j] - 1 - cj);
      const bool bnd = ((b.np >> j) & 1) && bj < 4;
      const double *wb = m->bwD[bnd ? bj + (n[j] - 1 - cj < cj ? 4 : 0) : 0];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double *f = P + (L::PU + i) * nS + s;
        double v[9];
#pragma unroll
        for (int o = 0; o < 9; ++o) v[o] = f[(o - 4) * st[j]];
        double g;
        if (bnd) {
          g = 0.0;
#pragma unroll
          for (int o = 0; o < 9; ++o) g += wb[o] * v[o];
          g *= b.idx[j];
        } else {
          g = d1(v, b.idx[j]);
        }
        G[(3 * j + i) * nS + s] = g;
      }
    }
  }
}

// Occupancy: two workgroups per CU (more spill, and the spills cost more than
// the extra waves gain), three for the reference-species x pass of up to 9
// species.
// REF: the reference-species form of the species diffusion (its own
// instance: the branch would otherwise raise the register use of both).
// WIDE: the second-derivative pairs with the wide stencil D(a D u) of two
// eighth-order first derivatives (Section 2.2) instead of the narrow one;
// its u samples reach 8 cells along D, taken from the periodic images.
// parts: bit 1 the convective terms, bit 2 the diffusive terms, bit 8 store
// the pass's sums into F instead of adding them (the first pass of an
// evaluation that nothing wrote to before).
// Physical boundaries along D (Section 2.5): the plain instances skip the
// cells within 4 of them; the BND instance runs on exactly those cells (its
// own work list) with the boundary stencils of the mechanism tables: first
// derivatives of the advective and of the diffusive terms, and the matrix K
// of the second-derivative pairs in place of the face-difference matrix B.
template <int NS, int D, bool FIXED, bool REF, bool WIDE, bool BND>
__global__ __launch_bounds__(256, D == 0 && NS <= 9 && REF && !WIDE && !BND ? 3 : 2) void k_dir(const BoxDev *__restrict__ boxes,
                                             const Item *__restrict__ items, int nitems,
                                             TileShape ts, FRef Uref,
                                             const double *__restrict__ Pbase,
                                             const double *__restrict__ Gbase, FRef Fout,
                                             unsigned parts, const DevMech *__restrict__ m,
                                             const int *__restrict__ skip) {
  if (skip && *skip) return;   // a residual early exit ended the step's sweeps
  using L = Layout<NS>;
  constexpr int NU = L::NU, NP = L::NP;
  constexpr int J1 = D == 0 ? 1 : 0, J2 = D == 2 ? 1 : 2;   // the two other directions
  // per-thread LDS column for the species centre values (up to 9 species:
  // 36 KiB per workgroup)
  constexpr bool SPEC_LDS = NS <= 9;
  __shared__ double spec_sh[SPEC_LDS ? 2 * NS * 256 : 1];
  // more species: their accumulators live in the thread's LDS column (a
  // register array indexed by the species loop would fall to scratch)
  constexpr bool ACC_LDS = !SPEC_LDS;
  __shared__ double acc_sh[ACC_LDS ? NS * 256 : 1];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int x, y, z;
    tile_cell(w, ts, x, y, z);
    if (x >= b.nx || y >= b.ny || z >= b.nz) continue;
    // cells within 4 of a physical boundary along D belong to the BND
    // instance; vb = its stencil variant (distance + 4 for the upper side)
    const int cD = D == 0 ? x : (D == 1 ? y : z), nDd = D == 0 ? b.nx : (D == 1 ? b.ny : b.nz);
    int vb = 0;
    if constexpr (BND) {
      // (the boundary work lists give every wave cells of one plane along D)
      vb = __builtin_amdgcn_readfirstlane(min(cD, nDd - 1 - cD) + (nDd - 1 - cD < cD ? 4 : 0));
    } else {
      if (((b.np >> D) & 1) && (cD < 4 || cD >= nDd - 4)) continue;
    }
    // per-lane cell indices are 32-bit; everything uniform (field bases,
    // stencil offsets) goes into the 64-bit base of each load
    const long long nS = (long long)b.sx * b.sy * b.sz;
    const long long nI = (long long)b.nx * b.ny * b.nz;
    const unsigned s = ((unsigned)(z + NSDC_NG) * b.sy + (y + NSDC_NG)) * b.sx + (x + NSDC_NG);
    const unsigned i = ((unsigned)z * b.ny + y) * b.nx + x;
    const long long st = D == 0 ? 1 : (D == 1 ? (long long)b.sx : (long long)b.sx * b.sy);
    const double *U = Uref.get(w.box, b.offS * NU);
    const double *P = Pbase + b.offS * NP;
    const double *G = Gbase + b.offS * 9;
    double *F = Fout.get(w.box, b.offI * NU);
    const double idx = b.idx[D], idx2 = b.idx2[D];
    // first derivatives of the advective (DA) and diffusive (DD) terms, of
    // a pointwise product (DAP, DDP), and v = B u (BV) for the pairs
    const double *wA = m->bwA[vb], *wD = m->bwD[vb];
    auto dotw = [&](const double *w, const double *f) {
      double r = 0.0;
#pragma unroll
      for (int o = 0; o < 9; ++o) r += w[o] * f[o];
      return r * idx;
    };
    auto dotwp = [&](const double *w, const double *f, const double *g) {
      double r = 0.0;
#pragma unroll
      for (int o = 0; o < 9; ++o) r += w[o] * (f[o] * g[o]);
      return r * idx;
    };
    auto DA = [&](const double *f) -> double {
      if constexpr (BND) return dotw(wA, f); else return d1(f, idx);
    };
    auto DD = [&](const double *f) -> double {
      if constexpr (BND) return dotw(wD, f); else return d1(f, idx);
    };
    auto DAP = [&](const double *f, const double *g) -> double {
      if constexpr (BND) return dotwp(wA, f, g); else return d1p(f, g, idx);
    };
    auto DDP = [&](const double *f, const double *g) -> double {
      if constexpr (BND) return dotwp(wD, f, g); else return d1p(f, g, idx);
    };
    auto BV = [&](const double *u, double *v) {
      if constexpr (BND) {
        const double(*K)[9] = m->bK[vb];
#pragma unroll
        for (int o = 0; o < 9; ++o) {
          double a = 0.0;
#pragma unroll
          for (int c = 0; c < 9; ++c) a += K[o][c] * u[c];
          v[o] = a;
        }
      } else {
        bvec<FIXED>(m, u, v);
      }
    };
    double acc[ACC_LDS ? 5 : NU];
#pragma unroll
    for (int q = 0; q < (ACC_LDS ? 5 : NU); ++q) acc[q] = 0.0;
    double *asp = acc_sh + threadIdx.x;
    if constexpr (ACC_LDS) {
#pragma unroll 1
      for (int k = 0; k < NS; ++k) asp[k * 256] = 0.0;
    }
    // species accumulator k
    auto spc = [&](int k) -> double & {
      if constexpr (ACC_LDS)
        return asp[k * 256];
      else
        return acc[5 + k];
    };
    auto line = [&](const double *f, double *v) {
      if constexpr (D == 0) {
#pragma unroll
        for (int o = 0; o < 9; ++o) v[o] = (f + (o - 4) * st)[s];
      } else {
        // strided taps as buffer loads: the lane offset is shared by the nine
        // taps and each tap's stride multiple rides in the scalar offset
        // (global loads would need a 64-bit address per tap); the range,
        // [f - 4 st, f + nS), holds every tap of every interior cell
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(f - 4 * st), (short)0, (unsigned)((nS + 4 * st) * 8), 0x00020000);
#pragma unroll
        for (int o = 0; o < 9; ++o)
          v[o] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)(s * 8u), (int)(o * st * 8), 0));
      }
    };
    // wide stencil: 17 samples along D (periodic images past the ghost
    // layers), and v_o = w_o (D u)_o / idx with w the first-derivative
    // weights, so that the pair (a, u) is dot9(a, v) idx2 as for B u
    auto line17 = [&](const double *f, double *w) {
      const int cD = D == 0 ? x : (D == 1 ? y : z), nDim = D == 0 ? b.nx : (D == 1 ? b.ny : b.nz);
#pragma unroll
      for (int o = 0; o < 17; ++o) {
        const int c = ((cD + o - 8) % nDim + nDim) % nDim;
        w[o] = f[(long long)s + (long long)(c - cD) * st];
      }
    };
    auto wvec = [&](const double *w, double *v) {
      constexpr double W[9] = {-C4, -C3, -C2, -C1, 0.0, C1, C2, C3, C4};
#pragma unroll
      for (int o = 0; o < 9; ++o) {
        double du = 0.0;
#pragma unroll
        for (int c = 0; c < 9; ++c) du += W[c] * w[o + c];
        v[o] = W[o] * du;
      }
    };
    double ud[9], pp[9];
    line(P + (L::PU + D) * nS, ud);
    line(P + L::PP * nS, pp);

    // with the diffusive terms on, the species convective terms of the y and
    // z passes join the species diffusion loop (more independent loads per
    // iteration; along x the extra live registers spill); above nine species
    // (correction velocity) they join the last species loop of every pass,
    // as D_D(Y_k rho u_D) from the Y_k lines that loop loads anyway
    constexpr bool CONV_IN_LAST = !SPEC_LDS && !REF;
    constexpr bool HYP_IN_SPECIES = D != 0 && !CONV_IN_LAST;
    const bool hyp_species_apart = CONV_IN_LAST ? (parts & 2) == 0 : (!HYP_IN_SPECIES || (parts & 2) == 0);
    if (parts & 1) {  // convective terms -D_D(F_D(U))
      double f[9];
#pragma unroll
      for (int ic = 0; ic < 3; ++ic) {
        line(U + (1 + ic) * nS, f);
        if (ic == D) acc[0] -= DA(f);
#pragma unroll
        for (int o = 0; o < 9; ++o) f[o] = f[o] * ud[o] + (ic == D ? pp[o] : 0.0);
        acc[1 + ic] -= DA(f);
      }
      line(U + 4 * nS, f);
#pragma unroll
      for (int o = 0; o < 9; ++o) f[o] += pp[o];
      acc[4] -= DAP(f, ud);
      if (hyp_species_apart) {
#pragma unroll 1
        for (int k = 0; k < NS; ++k) {
          line(U + (5 + k) * nS, f);
          spc(k) -= DAP(f, ud);
        }
      }
    }

    if (parts & 2) {  // diffusive terms
      const double bulk = m->bulk;
      const double lam2 = bulk - 2.0 / 3.0;
      // X_k lines formed from the Y_k lines and the mean molecular weight
      // (the same bits as the stored X_k, one line fewer per species), and
      // h_k lines from the temperature line (h_k = R_k (T p_k(T) + a6_k), p_k
      // the enthalpy polynomial); the temperature line, loaded once, also
      // serves the heat conduction
      constexpr bool XLINE = !WIDE && !REF;
      constexpr bool HLINE = XLINE;
      double T9[HLINE ? 9 : 1];
      if constexpr (WIDE) {
        // the same terms with the wide pairs
        double mu[9], ke[17], fe[9], w[17], v[9], g[9];
        line(P + L::PMU * nS, mu);
#pragma unroll
        for (int o = 0; o < 17; ++o) ke[o] = 0.0;
#pragma unroll
        for (int o = 0; o < 9; ++o) fe[o] = 0.0;
#pragma unroll
        for (int ic = 0; ic < 3; ++ic) {
          line17(P + (L::PU + ic) * nS, w);
          const double *u9 = w + 4;
          wvec(w, v);
          acc[1 + ic] += (ic == D ? 4.0 / 3.0 + bulk : 1.0) * dot9(mu, v) * idx2;
#pragma unroll
          for (int o = 0; o < 17; ++o) ke[o] += 0.5 * w[o] * w[o];
          if (ic == D) {
            line(G + (3 * J1 + J1) * nS, g);
            line(G + (3 * J2 + J2) * nS, v);
#pragma unroll
            for (int o = 0; o < 9; ++o) {
              g[o] = lam2 * mu[o] * (g[o] + v[o]);
              fe[o] += u9[o] * g[o];
            }
            acc[1 + D] += DD(g);
            double w2[17];
#pragma unroll
            for (int o = 0; o < 17; ++o) w2[o] = 0.5 * w[o] * w[o];
            wvec(w2, v);
            acc[4] += (1.0 / 3.0 + bulk) * dot9(mu, v) * idx2;
          } else {
            line(G + (3 * ic + D) * nS, g);
#pragma unroll
            for (int o = 0; o < 9; ++o) {
              g[o] *= mu[o];
              fe[o] += u9[o] * g[o];
            }
            acc[1 + ic] += DD(g);
          }
        }
        wvec(ke, v);
        acc[4] += dot9(mu, v) * idx2 + DD(fe);
        line17(P + L::PT * nS, w);
        wvec(w, v);
        line(P + L::PLAM * nS, g);
        acc[4] += dot9(g, v) * idx2;
      } else {
        double mu[9], ke[9], fe[9], u9[9], v[9], g[9];
        line(P + L::PMU * nS, mu);
#pragma unroll
        for (int o = 0; o < 9; ++o) ke[o] = fe[o] = 0.0;
#pragma unroll
        for (int ic = 0; ic < 3; ++ic) {
          if (ic == D) {
#pragma unroll
            for (int o = 0; o < 9; ++o) u9[o] = ud[o];
          } else {
            line(P + (L::PU + ic) * nS, u9);
          }
          // viscous stress, second-derivative part: L_D(a, u_ic),
          // a = (4/3 mu + xi) along D, mu across
          BV(u9, v);
          acc[1 + ic] += (ic == D ? 4.0 / 3.0 + bulk : 1.0) * dot9(mu, v) * idx2;
#pragma unroll
          for (int o = 0; o < 9; ++o) ke[o] += 0.5 * u9[o] * u9[o];
          if (ic == D) {
            // D_D((xi - 2/3 mu) sum_{j!=D} D_j u_j) and its viscous-work part
            line(G + (3 * J1 + J1) * nS, g);
            line(G + (3 * J2 + J2) * nS, v);
#pragma unroll
            for (int o = 0; o < 9; ++o) {
              g[o] = lam2 * mu[o] * (g[o] + v[o]);
              fe[o] += u9[o] * g[o];
            }
            acc[1 + D] += DD(g);
            // viscous work L_D(mu/3 + xi, u_D^2 / 2)
#pragma unroll
            for (int o = 0; o < 9; ++o) g[o] = 0.5 * u9[o] * u9[o];
            BV(g, v);
            acc[4] += (1.0 / 3.0 + bulk) * dot9(mu, v) * idx2;
          } else {
            // D_D(mu D_ic u_D) and its viscous-work part mu u_ic D_ic u_D
            line(G + (3 * ic + D) * nS, g);
#pragma unroll
            for (int o = 0; o < 9; ++o) {
              g[o] *= mu[o];
              fe[o] += u9[o] * g[o];
            }
            acc[1 + ic] += DD(g);
          }
        }
        // viscous work L_D(mu, |u|^2/2) and the first-derivative part
        BV(ke, v);
        acc[4] += dot9(mu, v) * idx2 + DD(fe);
        // heat conduction L_D(lambda, T)
        if constexpr (HLINE) {
          line(P + L::PT * nS, T9);
          BV(T9, v);
        } else {
          line(P + L::PT * nS, u9);
          BV(u9, v);
        }
        line(P + L::PLAM * nS, g);
        acc[4] += dot9(g, v) * idx2;
      }
      // species diffusion (pairs (rho D_k, X_k), (rho D_k (X_k-Y_k)/p, p) and
      // the energy pairs with h_k) and the correction velocity V_c,D, div V_c
      {
        double rd[9], wp[9], u9[9], v[9], g[9], wb9[XLINE ? 9 : 1];
        line(P + L::PRD * nS, rd);
        if constexpr (XLINE) line(P + L::PWB * nS, wb9);
        auto hline = [&](int k, double *h) {
          if constexpr (HLINE) {
            const double *c = m->hc[k];
            const double rk = m->Rk[k], a6 = m->h6[k];
#pragma unroll
            for (int o = 0; o < 9; ++o) {
              const double T = T9[o];
              h[o] = rk * fma(T, c[0] + T * (c[1] + T * (c[2] + T * (c[3] + T * c[4]))), a6);
            }
          } else {
            line(P + (L::PH + k) * nS, h);
          }
        };
        if constexpr (WIDE) {
          double w[17];
          line17(P + L::PP * nS, w);
          wvec(w, v);
        } else {
          BV(pp, v);
        }
        // X_k's centre samples into u9 and its pair vector into v
        auto xpair = [&](const double *f, double *u9o, double *vo) {
          if constexpr (WIDE) {
            double w[17];
            line17(f, w);
#pragma unroll
            for (int o = 0; o < 9; ++o) u9o[o] = w[o + 4];
            wvec(w, vo);
          } else {
            line(f, u9o);
            BV(u9o, vo);
          }
        };
#pragma unroll
        for (int o = 0; o < 9; ++o) wp[o] = rd[o] * v[o] / pp[o];
        const double Dpp = DD(pp) / pp[4];
        const double rd4 = rd[4];
        double divVc = 0.0, Vc = 0.0;
        if constexpr (REF) {
          const int ref = m->ref;
          // reference species (Section 2.1): species k != ref take their
          // mixture-model flux terms, the reference species minus their sum;
          // the energy pairs carry h_k - h_ref (Section 2.4); no V_c terms
          double tsum = 0.0;
#pragma unroll 1
          for (int k = 0; k < NS; ++k) {
            if (HYP_IN_SPECIES && (parts & 1)) {
              line(U + (5 + k) * nS, u9);
              spc(k) -= DAP(u9, ud);
            }
            if (k == ref) continue;
            const double iLe = m->invLe[k];
            xpair(P + (L::PX + k) * nS, u9, v);
            line(P + (L::PY + k) * nS, g);
#pragma unroll
            for (int o = 0; o < 9; ++o) u9[o] -= g[o];
            const double Lp = dot9(u9, wp);
            const double Lx = dot9(rd, v);
            line(P + (L::PH + k) * nS, g);
            {
              double hr[9];
              line(P + (L::PH + ref) * nS, hr);
#pragma unroll
              for (int o = 0; o < 9; ++o) g[o] -= hr[o];
            }
            double LhX = 0.0, Lpe = 0.0;
#pragma unroll
            for (int o = 0; o < 9; ++o) {
              LhX += rd[o] * g[o] * v[o];
              Lpe += u9[o] * g[o] * wp[o];
            }
            const double t = iLe * (Lx + Lp) * idx2;
            spc(k) += t;
            tsum += t;
            acc[4] += iLe * (LhX + Lpe) * idx2;
          }
          if constexpr (ACC_LDS) {
            spc(ref) -= tsum;
          } else {
#pragma unroll
            for (int k = 0; k < NS; ++k)
              if (k == ref) spc(k) -= tsum;
          }
        } else if constexpr (SPEC_LDS) {
          // one pass over the species lines: the centre values Y_k and first
          // derivatives D_D Y_k of the final Y_k div V_c + V_c D_D Y_k terms
          // wait in this thread's LDS column; the energy counterpart is
          // summed over species as it goes
          double *ysh = spec_sh + threadIdx.x;
          double ShY = 0.0, SDhY = 0.0;
#pragma unroll 1
          for (int k = 0; k < NS; ++k) {
            const double iLe = m->invLe[k];
            double y9[9];
            if (HYP_IN_SPECIES && (parts & 1)) {
              line(U + (5 + k) * nS, y9);
              spc(k) -= DAP(y9, ud);
            }
            if constexpr (WIDE) {
              xpair(P + (L::PX + k) * nS, u9, v);
              line(P + (L::PY + k) * nS, y9);
              line(P + (L::PH + k) * nS, g);
            } else {
              // X_k = Y_k Wbar / W_k as the primitives kernel forms it
              line(P + (L::PY + k) * nS, y9);
              hline(k, g);
#pragma unroll
              for (int o = 0; o < 9; ++o) u9[o] = y9[o] * wb9[o] * m->invW[k];
              BV(u9, v);
            }
            const double DX = DD(u9);
            const double dXY4 = u9[4] - y9[4];
#pragma unroll
            for (int o = 0; o < 9; ++o) u9[o] -= y9[o];
            const double Lp = dot9(u9, wp);
            const double Lx = dot9(rd, v);
            double LhX = 0.0, Lpe = 0.0;
#pragma unroll
            for (int o = 0; o < 9; ++o) {
              LhX += rd[o] * g[o] * v[o];
              Lpe += u9[o] * g[o] * wp[o];
            }
            const double t = iLe * (Lx + Lp) * idx2;
            spc(k) += t;
            divVc -= t;
            acc[4] += iLe * (LhX + Lpe) * idx2;
            Vc -= rd4 * iLe * (DX + dXY4 * Dpp);
            ysh[k * 256] = y9[4];
            ysh[(NS + k) * 256] = DD(y9);
            ShY += g[4] * y9[4];
            SDhY += DDP(g, y9);
          }
          // Y_k (div V_c)_D + V_c,D D_D Y_k and the energy counterpart
#pragma unroll
          for (int k = 0; k < NS; ++k) spc(k) += ysh[k * 256] * divVc + Vc * ysh[(NS + k) * 256];
          acc[4] += ShY * divVc + Vc * SDhY;
        } else {
#pragma unroll 1
          for (int k = 0; k < NS; ++k) {
            const double iLe = m->invLe[k];
            if (HYP_IN_SPECIES && (parts & 1)) {
              line(U + (5 + k) * nS, u9);
              spc(k) -= DAP(u9, ud);
            }
            if constexpr (!XLINE) {
              xpair(P + (L::PX + k) * nS, u9, v);
              line(P + (L::PY + k) * nS, g);
            } else {
              // X_k = Y_k Wbar / W_k as the primitives kernel forms it
              line(P + (L::PY + k) * nS, g);
#pragma unroll
              for (int o = 0; o < 9; ++o) u9[o] = g[o] * wb9[o] * m->invW[k];
              BV(u9, v);
            }
            const double DX = DD(u9);
            const double dXY4 = u9[4] - g[4];
#pragma unroll
            for (int o = 0; o < 9; ++o) u9[o] -= g[o];
            const double Lp = dot9(u9, wp);
            const double Lx = dot9(rd, v);
            hline(k, g);
            double LhX = 0.0, Lpe = 0.0;
#pragma unroll
            for (int o = 0; o < 9; ++o) {
              LhX += rd[o] * g[o] * v[o];
              Lpe += u9[o] * g[o] * wp[o];
            }
            const double t = iLe * (Lx + Lp) * idx2;
            spc(k) += t;
            divVc -= t;
            acc[4] += iLe * (LhX + Lpe) * idx2;
            Vc -= rd4 * iLe * (DX + dXY4 * Dpp);
          }
          // Y_k (div V_c)_D + V_c,D D_D Y_k and the energy counterpart with
          // h_k Y_k, and the convective terms with the momentum line along D
          // (loaded again here: the barrier keeps the compiler from holding
          // the convective part's copy live through the pass)
          double m9[9];
          if (parts & 1) {
            asm volatile("" ::: "memory");
            line(U + (1 + D) * nS, m9);
          }
#pragma unroll 1
          for (int k = 0; k < NS; ++k) {
            line(P + (L::PY + k) * nS, u9);
            hline(k, g);
            const double DY = DD(u9);
            const double DhY = DDP(g, u9);
            double sk = u9[4] * divVc + Vc * DY;
            if (parts & 1) sk -= DAP(u9, m9);
            spc(k) += sk;
            acc[4] += g[4] * u9[4] * divVc + Vc * DhY;
          }
        }
      }
    }
    // the first pass of an evaluation that nothing wrote to before (bit 8
    // of parts) stores its sums; every other pass adds to what is there
    if (parts & 8) {
      if constexpr (ACC_LDS) {
#pragma unroll
        for (int q = 0; q < 5; ++q) (F + q * nI)[i] = acc[q];
#pragma unroll 1
        for (int k = 0; k < NS; ++k) (F + (5 + k) * nI)[i] = spc(k);
      } else {
#pragma unroll
        for (int q = 0; q < NU; ++q) (F + q * nI)[i] = acc[q];
      }
    } else {
      if constexpr (ACC_LDS) {
#pragma unroll
        for (int q = 0; q < 5; ++q) (F + q * nI)[i] += acc[q];
#pragma unroll 1
        for (int k = 0; k < NS; ++k) (F + (5 + k) * nI)[i] += spc(k);
      } else {
#pragma unroll
        for (int q = 0; q < NU; ++q) (F + q * nI)[i] += acc[q];
      }
    }
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
  NSDC_CHEM_LDS(NS, NSDC_CHEM_LDS_LIMIT, chem_sh);
  double *sh = chem_lds_setup<NS, NSDC_CHEM_LDS_LIMIT>(chem_sh, m);
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
    production_any<NS, NSDC_CHEM_LDS_LIMIT>(m, rho, T, Y, wd, sh);
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
                                                  NodeArgs a, const int *__restrict__ skip) {
  if (skip && *skip) return;   // a residual early exit ended the step's sweeps
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

// Residual of eq. (residual) after a sweep: per component the largest |R|,
// R = U_0 + dt sum_j q_j F_j - U_M, and the largest |U_0| over the interior
// cells of the workgroup's items (a grid of at most NSDC_RESID_BLOCKS
// workgroups), written to partial[block][2 NU]; maxima are independent of
// the order, so the result is deterministic.
template <int NS>
__global__ __launch_bounds__(256) void k_sdc_resid(const BoxDev *__restrict__ boxes,
                                                   const Item *__restrict__ items, int nitems,
                                                   TileShape ts, FRef U0ref, FRef UMref, ResidArgs a, const int *__restrict__ skip) {
  if (skip && *skip) return;   // a residual early exit ended the step's sweeps
  constexpr int NU = 5 + NS;
  __shared__ double red[256];
  double rmax[NU], umax[NU];
#pragma unroll
  for (int q = 0; q < NU; ++q) rmax[q] = umax[q] = 0.0;
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
    const double *U0 = U0ref.get(w.box, b.offS * NU);
    const double *UM = UMref.get(w.box, b.offS * NU);
#pragma unroll
    for (int q = 0; q < NU; ++q) {
      const long long qi = oI + q * nI + i;
      double sf = 0.0;
      for (int j = 0; j < a.nnodes; ++j) sf += a.q[j] * a.F[j][qi];
      const double u0 = U0[q * nS + s];
      rmax[q] = fmax(rmax[q], fabs(u0 + a.dt * sf - UM[q * nS + s]));
      umax[q] = fmax(umax[q], fabs(u0));
    }
  }
  const int t = threadIdx.x, nt = blockDim.x;
#pragma unroll
  for (int v = 0; v < 2 * NU; ++v) {
    red[t] = v < NU ? rmax[v] : umax[v - NU];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (t < h && t + h < nt) red[t] = fmax(red[t], red[t + h]);
      __syncthreads();
    }
    if (t == 0) a.partial[blockIdx.x * 2 * NU + v] = red[0];
    __syncthreads();
  }
}

// out[v] = max over the nblocks rows of partial[.][v]: workgroup v of ncol,
// 256 threads striding over the rows, then a tree in LDS.
__global__ __launch_bounds__(256) void k_rows_max(const double *__restrict__ partial, int nblocks, int ncol,
                                                  double *__restrict__ out,
                                                  const int *__restrict__ skip) {
  if (skip && *skip) return;   // a residual early exit ended the step's sweeps
  __shared__ double red[256];
  const int v = blockIdx.x, t = threadIdx.x;
  double m = 0.0;
  for (int b = t; b < nblocks; b += 256) m = fmax(m, partial[(long long)b * ncol + v]);
  red[t] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] = fmax(red[t], red[t + h]);
    __syncthreads();
  }
  if (t == 0) out[v] = red[0];
}

// One coarse interval of the multirate sweep, mode 1 (eq. mrupdate):
//   U_{q+1} = U_q + dtau_q [f1(U^{k+1}_p) - f1(U^k_p)] + dtau_q [f2(U^{k+1}_q) - f2(U^k_q)]
//             + dt S22_q . F2^k + dt S21_q . F1^k,
// f2 the chemistry (species components only).  Everything except the
// f2(U^{k+1}_q) term is known before the interval starts; k_mr_src forms it
// for all fine sub-steps of the interval (a streaming pass over the node
// values) into A[q][component], and k_mr_step then runs the sub-steps of a
// cell in registers: Newton, chemistry, U += A[q] + dtau_q f2.
template <int NS, int NQ>
__global__ __launch_bounds__(256) void k_mr_src(const BoxDev *__restrict__ boxes,
                                                const Item *__restrict__ items, int nitems,
                                                TileShape ts, const FineCoef *__restrict__ fc,
                                                FinePtrs fp, double *__restrict__ Abase,
                                                long long aslot) {
  constexpr int NU = 5 + NS;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int x, y, z;
    tile_cell(w, ts, x, y, z);
    if (x >= b.nx || y >= b.ny || z >= b.nz) continue;
    const long long nI = (long long)b.nx * b.ny * b.nz;
    const unsigned i = ((unsigned)z * b.ny + y) * b.nx + x;
    const long long o1 = b.offI * NU, o2 = b.offI * NS;
    auto F1 = [&](int slot, int q) { return fp.F1base + (slot * fp.f1slot + o1 + q * nI); };
    auto F2 = [&](int slot, int k) { return fp.F2base + (slot * fp.f2slot + o2 + k * nI); };
    auto A = [&](int r, int q) { return Abase + (r * aslot + o1 + q * nI); };
    const int n1 = fc->n1, nf = fc->nfine;
    const int nq = NQ > 0 ? NQ : fc->nq;
    const double dt = fp.dt;
#pragma unroll 1
    for (int q = 0; q < NU; ++q) {
      // coefficient tables are re-read per component (scalar loads) rather
      // than hoisted into more scalar registers than there are
      asm volatile("" ::: "memory");
      double f1[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) f1[j] = j < n1 ? F1(fp.F1old[j], q)[i] : 0.0;
      const double dF1 = F1(fp.F1new_p, q)[i] - F1(fp.F1old_p, q)[i];
      if (NQ > 0) {
        // NQ sub-steps: the interval's NQ + 1 fine-node values of this
        // species are loaded once, with every other operand, before any use
        double g[NQ + 1];
        if (q >= 5) {
#pragma unroll
          for (int j = 0; j <= NQ; ++j) g[j] = F2(fp.F2old[j], q - 5)[i];
        }
#pragma unroll
        for (int r = 0; r < NQ; ++r) {
          const double dtq = fc->dtq[r] * dt;
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < 8; ++j) acc += fc->S21[r][j] * f1[j];
          double v = dtq * dF1 + dt * acc;
          if (q >= 5) {
            const int jlo = fc->jlo[r];
            double s22 = 0.0;
#pragma unroll
            for (int j = 0; j <= NQ; ++j) {
              const int jj = j - jlo;   // position in the interpolating piece
              if (jj >= 0 && jj < nf) s22 += fc->S22[r][jj] * g[j];
            }
            v += dt * s22 - dtq * g[r];
          }
          A(r, q)[i] = v;
        }
      } else {
#pragma unroll 1
        for (int r = 0; r < nq; ++r) {
          const double dtq = fc->dtq[r] * dt;
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < 8; ++j) acc += fc->S21[r][j] * f1[j];
          double v = dtq * dF1 + dt * acc;
          if (q >= 5) {
            const int k = q - 5, jlo = fc->jlo[r];
            double s22 = 0.0;
#pragma unroll
            for (int j = 0; j < 9; ++j)
              if (j < nf) s22 += fc->S22[r][j] * F2(fp.F2old[jlo + j], k)[i];
            v += dt * s22 - dtq * F2(fp.F2old[r], k)[i];
          }
          A(r, q)[i] = v;
        }
      }
    }
  }
}

template <int NS>
__global__ __launch_bounds__(256) void k_mr_step(const BoxDev *__restrict__ boxes,
                                                 const Item *__restrict__ items, int nitems,
                                                 TileShape ts, FRef Uin, FRef Uout,
                                                 const FineCoef *__restrict__ fc, FinePtrs fp,
                                                 const double *__restrict__ Abase, long long aslot,
                                                 const DevMech *__restrict__ m, int *err) {
  constexpr int NU = 5 + NS;
  NSDC_CHEM_LDS(NS, NSDC_CHEM_LDS_LIMIT, chem_sh);
  double *sh = chem_lds_setup<NS, NSDC_CHEM_LDS_LIMIT>(chem_sh, m);
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int x, y, z;
    tile_cell(w, ts, x, y, z);
    if (x >= b.nx || y >= b.ny || z >= b.nz) continue;
    const long long nS = (long long)b.sx * b.sy * b.sz, nI = (long long)b.nx * b.ny * b.nz;
    const unsigned s = ((unsigned)(z + NSDC_NG) * b.sy + (y + NSDC_NG)) * b.sx + (x + NSDC_NG);
    const unsigned i = ((unsigned)z * b.ny + y) * b.nx + x;
    const long long o1 = b.offI * NU, o2 = b.offI * NS;
    auto F2 = [&](int slot, int k) { return fp.F2base + (slot * fp.f2slot + o2 + k * nI); };
    auto A = [&](int r, int q) { return Abase + (r * aslot + o1 + q * nI); };
    const double *Ui = Uin.get(w.box, b.offS * NU);
    double *Uo = Uout.get(w.box, b.offS * NU);
    double Uc[NU];
#pragma unroll
    for (int q = 0; q < NU; ++q) Uc[q] = (Ui + q * nS)[s];
    const int nq = fc->nq;
    int errs = 0;
    // the temperature of the previous sub-step seeds the next Newton solve
    double Tprev = 1000.0;
    for (int qq = 0; qq < nq; ++qq) {
      double f2[NS];
      if (qq == 0 && fp.q0_known) {
#pragma unroll
        for (int k = 0; k < NS; ++k) f2[k] = F2(fp.F2old[0], k)[i];
      } else {
        double rho, u[3], Y[NS], T;
        errs |= cell_state<NS>(m, Uc, rho, u, Y, T, Tprev);
        Tprev = T;
        production_any<NS, NSDC_CHEM_LDS_LIMIT>(m, rho, T, Y, f2, sh);
#pragma unroll
        for (int k = 0; k < NS; ++k) F2(fp.F2new[qq], k)[i] = f2[k];
      }
      const double dtq = fc->dtq[qq] * fp.dt;
#pragma unroll
      for (int q = 0; q < NU; ++q) Uc[q] += A(qq, q)[i] + (q >= 5 ? dtq * f2[q - 5] : 0.0);
    }
    if (fp.eval_last) {
      double rho, u[3], Y[NS], T, f2[NS];
      errs |= cell_state<NS>(m, Uc, rho, u, Y, T, Tprev);
      production_any<NS, NSDC_CHEM_LDS_LIMIT>(m, rho, T, Y, f2, sh);
#pragma unroll
      for (int k = 0; k < NS; ++k) F2(fp.F2new[nq], k)[i] = f2[k];
    }
    if (errs) atomicOr(err, errs);
#pragma unroll
    for (int q = 0; q < NU; ++q) (Uo + q * nS)[s] = Uc[q];
  }
}

// Orders the LDS accesses of the lanes of one wave (the two lanes that share
// a cell's slot in the two-lane implicit chemistry kernel are in one wave; a
// wave executes its LDS instructions in issue order, so only the compiler
// must not move them).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane pairs for more than nine species: a cell's chemistry arrays in LDS
// (b_k and two production arrays: 3 (Ns+1) doubles, 528 bytes at 21 species)
// would allow one wave per SIMD with a lane per cell; two lanes sharing a
// cell's column halve the LDS per lane, so two waves per SIMD fit.  The two
// lanes of a cell are lane l of the two waves of a 128-thread workgroup
// (cell slot l; a workgroup per pair of waves, so that the pair's barriers
// hold no other waves): the lane's half, sub = its wave, is uniform over a
// wave, so the species and reactions a lane takes are the
// same for its whole wave and their coefficients come from scalar loads of
// the mechanism.  Each lane sums its reactions' contributions into its own
// production array, in reaction order, and the two arrays are added in a
// fixed order, so the result does not depend on how the two waves
// interleave.  The pair's exchanges through LDS synchronise the workgroup,
// so every thread runs every pass of the cell loop (lanes without a cell
// compute on the tile's first cell and store nothing).
struct PairLane {
  int sub, slot;
  __device__ PairLane() {
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    sub = wv & 1;
    slot = (wv >> 1) * 64 + (int)(threadIdx.x & 63);
  }
};

// Lane SUB's reactions j = SUB, SUB + 2, ...: their rates of progress
// (production()'s form) added into its production array (offset (1 + SUB) A
// of the column; b_k at offset 0).
template <int NS, int CS, int SUB>
__device__ __forceinline__ void pair_loop(const DevMech *__restrict__ m, double T, double invT, double lnT,
                                          double *sh, const double *tab) {
  constexpr int A = (NS + 1) * CS, WO = (1 + SUB) * A;
  const int nr = m->nr;
#pragma unroll 4
  for (int j = SUB; j < nr; j += 2) {
    const int r0 = m->rs[j][0] * CS, r1 = m->rs[j][1] * CS, p0 = m->ps[j][0] * CS, p1 = m->ps[j][1] * CS;
    const double q = exp_tab(rate_exponent(m, j, T, invT, lnT), tab) * (sh[r0] * sh[r1] - sh[p0] * sh[p1]);
    atomicAdd(sh + WO + r0, -q);
    atomicAdd(sh + WO + r1, -q);
    atomicAdd(sh + WO + p0, q);
    atomicAdd(sh + WO + p1, q);
  }
}

// The chemistry source of one cell on a lane pair: the pair's LDS column sh
// holds b_k and the lanes' production arrays at offsets 0, A and 2 A, slot k
// at k CS.  Lane sub sets up the slots k = sub, sub + 2, ... (the dummy slot
// NS included, so the pair forms each exponential b_k once), clears its
// production array and takes its reactions.  Every thread of the workgroup
// calls it; on return the cell's production of slot k is
// sh[A + k CS] + sh[2 A + k CS].
template <int NS, int CS>
__device__ __forceinline__ void pair_rates(const DevMech *__restrict__ m, double rho, double T, const double *Yo,
                                           double *sh, int sub, const double *tab) {
  constexpr int A = (NS + 1) * CS, NK = (NS + 1) / 2;
  const double lnT = log(T), invT = 1.0 / T, lnRTp = lnT + LN_RU_PREF;
  __syncthreads();   // the previous readers of the columns are done
#pragma unroll
  for (int n = 0; n < (NS + 2) / 2; ++n) {
    const int k0 = 2 * n, k1 = 2 * n + 1;
    if (k1 <= NS || sub == 0) {
      const int k = k0 + sub;
      const double y = Yo[n < NK ? n : NK - 1];
      sh[k * CS] = k < NS ? rho * y * m->invW[k] * exp_tab(g_RT(m, k, T, invT, lnT), tab) : exp_tab(-lnRTp, tab);
    }
  }
  double *wo = sh + (1 + sub) * A;
#pragma unroll
  for (int k = 0; k <= NS; ++k) wo[k * CS] = 0.0;
  __syncthreads();
  if (sub == 0)
    pair_loop<NS, CS, 0>(m, T, invT, lnT, sh, tab);
  else
    pair_loop<NS, CS, 1>(m, T, invT, lnT, sh, tab);
  __syncthreads();
}

// The cell of pass h (a multiple of 64) of a work item for pair slot `slot`:
// false (and the tile's first cell, which every work item has) when the slot
// has no cell in this pass.
__device__ __forceinline__ bool pair_cell(const Item &w, const BoxDev &b, const TileShape &ts, int h, int slot,
                                          unsigned &s, unsigned &i) {
  const int cell = h + slot;
  int x = w.x0 + cell % ts.tx, y = w.y0 + (cell / ts.tx) % ts.ty, z = w.z0 + cell / (ts.tx * ts.ty);
  const bool valid = cell < ts.tx * ts.ty * ts.tz && x < b.nx && y < b.ny && z < b.nz;
  if (!valid) {
    x = w.x0;
    y = w.y0;
    z = w.z0;
  }
  s = ((unsigned)(z + NSDC_NG) * b.sy + (y + NSDC_NG)) * b.sx + (x + NSDC_NG);
  i = ((unsigned)z * b.ny + y) * b.nx + x;
  return valid;
}

// k_mr_step on lane pairs (above): both lanes of a pair run the cell's state
// update and Newton solve (redundantly, same values) and split the species
// setup and the reactions (pair_rates); each lane writes half of the outputs.
// Launched with 128 threads whatever the tile: 64 cells per pass.
template <int NS>
__global__ __launch_bounds__(128, 2) void k_mr_pair(const BoxDev *__restrict__ boxes,
                                                    const Item *__restrict__ items, int nitems,
                                                    TileShape ts, FRef Uin, FRef Uout,
                                                    const FineCoef *__restrict__ fc, FinePtrs fp,
                                                    const double *__restrict__ Abase, long long aslot,
                                                    const DevMech *__restrict__ m, int *err) {
  constexpr int NU = 5 + NS, CS = 64, A = (NS + 1) * CS;
  __shared__ double col[3 * A];
  __shared__ double tab[64];
  for (int j = threadIdx.x; j < 64; j += blockDim.x) tab[j] = m->e2tab[j];
  const PairLane pl;
  const int sub = pl.sub;
  double *sh = col + pl.slot;
  // the chemistry source of one cell, rates split between the two lanes
  auto production_pair = [&](double rho, double T, const double *Y, double *wdot) {
    double Yo[(NS + 1) / 2];
#pragma unroll
    for (int n = 0; n < (NS + 1) / 2; ++n) Yo[n] = sub ? Y[2 * n + 1 < NS ? 2 * n + 1 : NS - 1] : Y[2 * n];
    pair_rates<NS, CS>(m, rho, T, Yo, sh, sub, tab);
#pragma unroll
    for (int k = 0; k < NS; ++k) wdot[k] = (sh[A + k * CS] + sh[2 * A + k * CS]) * m->W[k];
  };
  const int tcells = ts.tx * ts.ty * ts.tz;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    const long long nS = (long long)b.sx * b.sy * b.sz, nI = (long long)b.nx * b.ny * b.nz;
    const long long o1 = b.offI * NU, o2 = b.offI * NS;
    const double *Ui = Uin.get(w.box, b.offS * NU);
    double *Uo = Uout.get(w.box, b.offS * NU);
    auto F2 = [&](int slot, int k) { return fp.F2base + (slot * fp.f2slot + o2 + k * nI); };
    auto Af = [&](int r, int q) { return Abase + (r * aslot + o1 + q * nI); };
    for (int h = 0; h < tcells; h += CS) {
      unsigned s, i;
      const bool valid = pair_cell(w, b, ts, h, pl.slot, s, i);
      double Uc[NU];
#pragma unroll
      for (int q = 0; q < NU; ++q) Uc[q] = (Ui + q * nS)[s];
      const int nq = fc->nq;
      int errs = 0;
      double Tprev = 1000.0;
      for (int qq = 0; qq < nq; ++qq) {
        double f2[NS];
        if (qq == 0 && fp.q0_known) {
#pragma unroll
          for (int k = 0; k < NS; ++k) f2[k] = F2(fp.F2old[0], k)[i];
        } else {
          double rho, u[3], Y[NS], T;
          errs |= cell_state_pair<NS>(m, Uc, rho, u, Y, T, Tprev);
          Tprev = T;
          production_pair(rho, T, Y, f2);
          if (valid)
#pragma unroll
            for (int k = 0; k < NS; ++k)
              if ((k & 1) == sub) F2(fp.F2new[qq], k)[i] = f2[k];
        }
        const double dtq = fc->dtq[qq] * fp.dt;
#pragma unroll
        for (int q = 0; q < NU; ++q) Uc[q] += Af(qq, q)[i] + (q >= 5 ? dtq * f2[q - 5] : 0.0);
      }
      if (fp.eval_last) {
        double rho, u[3], Y[NS], T, f2[NS];
        errs |= cell_state_pair<NS>(m, Uc, rho, u, Y, T, Tprev);
        production_pair(rho, T, Y, f2);
        if (valid)
#pragma unroll
          for (int k = 0; k < NS; ++k)
            if ((k & 1) == sub) F2(fp.F2new[nq], k)[i] = f2[k];
      }
      if (!valid) continue;
      if (errs) atomicOr(err, errs);
#pragma unroll
      for (int q = 0; q < NU; ++q)
        if ((q & 1) == sub) (Uo + q * nS)[s] = Uc[q];
    }
  }
}

// k_mr_src and k_mr_pair in one kernel for four coarse nodes and four fine
// sub-steps above nine species: the increments of eq. (mrupdate) are formed in
// registers with k_mr_src's arithmetic and consumed by k_mr_pair's sub-steps,
// so they never reach HBM.  The lanes of a pair split the species: lane sub
// owns the species k with k mod 2 = sub, their 4 increments and partial
// densities; both lanes run the five non-species components through the
// sub-steps (their increments need only f1).  Before every temperature solve
// each lane sums the mixture's energy coefficients over its own species and
// the pair exchanges the two partial sums through the cell's LDS column, so
// both lanes solve with the same coefficients and operations as k_mr_pair
// (cell_state_pair): the results equal the two-kernel form bit for bit.
// Launched with 128 threads whatever the tile.
template <int NS>
__global__ __launch_bounds__(128, 2) void k_mr_pair_fused(const BoxDev *__restrict__ boxes,
                                                          const Item *__restrict__ items, int nitems,
                                                          TileShape ts, FRef Uin, FRef Uout,
                                                          const FineCoef *__restrict__ fc, FinePtrs fp,
                                                          const DevMech *__restrict__ m, int *err) {
  constexpr int NU = 5 + NS, CS = 64, A = (NS + 1) * CS, NQ = 4, N1 = 4;
  constexpr int NK = (NS + 1) / 2;   // species per lane (the even lane one more for odd NS)
  __shared__ double col[3 * A];
  __shared__ double tab[64];
  for (int j = threadIdx.x; j < 64; j += blockDim.x) tab[j] = m->e2tab[j];
  const PairLane pl;
  const int sub = pl.sub;
  double *sh = col + pl.slot;
  // as in k_mr_pair
  auto production_pair = [&](double rho, double T, const double *Y, double *wdot) {
    pair_rates<NS, CS>(m, rho, T, Y, sh, sub, tab);
    // this lane's species only
#pragma unroll
    for (int n = 0; n < NK; ++n) {
      const int k = 2 * n + sub;
      if (k < NS) wdot[n] = (sh[A + k * CS] + sh[2 * A + k * CS]) * m->W[k];
    }
  };
  const int tcells = ts.tx * ts.ty * ts.tz;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    const long long nS = (long long)b.sx * b.sy * b.sz, nI = (long long)b.nx * b.ny * b.nz;
    const long long o1 = b.offI * NU, o2 = b.offI * NS;
    const double *Ui = Uin.get(w.box, b.offS * NU);
    double *Uo = Uout.get(w.box, b.offS * NU);
    auto F1 = [&](int sl, int q) { return fp.F1base + (sl * fp.f1slot + o1 + q * nI); };
    auto F2 = [&](int sl, int k) { return fp.F2base + (sl * fp.f2slot + o2 + k * nI); };
    const double dt = fp.dt;
    for (int h = 0; h < tcells; h += CS) {
      unsigned s, i;
      const bool valid = pair_cell(w, b, ts, h, pl.slot, s, i);
      // increments of component q for the NQ sub-steps, k_mr_src's arithmetic
      // (four coarse nodes: k_mr_src's sums without its zero terms; the S22
      // rows padded with zeros to the interval's five fine nodes add exact
      // zeros)
      auto increments = [&](int q, double *inc) {
        asm volatile("" ::: "memory");
        double f1[N1];
#pragma unroll
        for (int j = 0; j < N1; ++j) f1[j] = F1(fp.F1old[j], q)[i];
        const double dF1 = F1(fp.F1new_p, q)[i] - F1(fp.F1old_p, q)[i];
        double g[NQ + 1];
        if (q >= 5) {
#pragma unroll
          for (int j = 0; j <= NQ; ++j) g[j] = F2(fp.F2old[j], q - 5)[i];
        }
#pragma unroll
        for (int r = 0; r < NQ; ++r) {
          const double dtq = fc->dtq[r] * dt;
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < N1; ++j) acc += fc->S21[r][j] * f1[j];
          double v = dtq * dF1 + dt * acc;
          if (q >= 5) {
            double s22 = 0.0;
#pragma unroll
            for (int j = 0; j <= NQ; ++j) s22 += fc->S22n[r][j] * g[j];
            v += dt * s22 - dtq * g[r];
          }
          inc[r] = v;
        }
      };
      // the non-species components through the sub-steps (the chemistry
      // leaves them alone): keep the density and internal energy each
      // temperature solve needs, formed as cell_state forms them, and the
      // final values
      double Un[5], rho_r[NQ + 1], e_r[NQ + 1];
      {
        double An[NQ][5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          Un[q] = (Ui + q * nS)[s];
          double inc[NQ];
          increments(q, inc);
#pragma unroll
          for (int r = 0; r < NQ; ++r) An[r][q] = inc[r];
        }
#pragma unroll
        for (int r = 0; r <= NQ; ++r) {
          rho_r[r] = Un[0];
          const double ir = 1.0 / Un[0];
          const double u0 = Un[1] * ir, u1 = Un[2] * ir, u2 = Un[3] * ir;
          e_r[r] = Un[4] * ir - 0.5 * (u0 * u0 + u1 * u1 + u2 * u2);
          if (r < NQ)
#pragma unroll
            for (int q = 0; q < 5; ++q) Un[q] += An[r][q] + 0.0;
        }
      }
      double Uk[NK], Ak[NQ][NK];
#pragma unroll
      for (int n = 0; n < NK; ++n) {
        const int k = 2 * n + sub;
        if (k < NS) {
          Uk[n] = (Ui + (5 + k) * nS)[s];
          double inc[NQ];
          increments(5 + k, inc);
#pragma unroll
          for (int r = 0; r < NQ; ++r) Ak[r][n] = inc[r];
        } else {
          Uk[n] = 0.0;
#pragma unroll
          for (int r = 0; r < NQ; ++r) Ak[r][n] = 0.0;
        }
      }
      // the temperature solve of sub-step r as cell_state_pair does it; Yo[n]
      // = Y of this lane's species 2 n + sub
      auto state = [&](int r, double &rho, double *Yo, double &T, double T0) {
        rho = rho_r[r];
        const double ir = 1.0 / rho;
#pragma unroll
        for (int n = 0; n < NK; ++n) Yo[n] = Uk[n] * ir;
        // e_coeffs over this lane's species k = 2 n + sub, in increasing k
        double p[6], c[6];
        asm volatile("" ::: "memory");
#pragma unroll
        for (int q = 0; q < 6; ++q) p[q] = 0.0;
#pragma unroll
        for (int n = 0; n < NK; ++n) {
          const int k = 2 * n + sub;
          if (k < NS) {
            const double YR = Yo[n] * m->Rk[k];
            const double *a = m->hc[k];
            p[0] += YR * (a[0] - 1.0);
            p[1] += YR * a[1];
            p[2] += YR * a[2];
            p[3] += YR * a[3];
            p[4] += YR * a[4];
            p[5] += YR * m->h6[k];
          }
        }
        __syncthreads();   // the previous readers of the columns are done
#pragma unroll
        for (int q = 0; q < 6; ++q) sh[(6 * sub + q) * CS] = p[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const double o = sh[(6 * (1 - sub) + q) * CS];
          c[q] = sub == 0 ? p[q] + o : o + p[q];
        }
        int e = rho > 0.0 ? 0 : NSDC_ERR_RHO;
        e |= temperature_c(m, c, e_r[r], T, T0);
        return e;
      };
      int errs = 0;
      double Tprev = 1000.0;
      for (int qq = 0; qq < NQ; ++qq) {
        double f2[NK];
        if (qq == 0 && fp.q0_known) {
#pragma unroll
          for (int n = 0; n < NK; ++n)
            if (2 * n + sub < NS) f2[n] = F2(fp.F2old[0], 2 * n + sub)[i];
        } else {
          double rho, Yo[NK], T;
          errs |= state(qq, rho, Yo, T, Tprev);
          Tprev = T;
          production_pair(rho, T, Yo, f2);
          if (valid)
#pragma unroll
            for (int n = 0; n < NK; ++n)
              if (2 * n + sub < NS) F2(fp.F2new[qq], 2 * n + sub)[i] = f2[n];
        }
        const double dtq = fc->dtq[qq] * dt;
#pragma unroll
        for (int n = 0; n < NK; ++n)
          if (2 * n + sub < NS) Uk[n] += Ak[qq][n] + dtq * f2[n];
      }
      if (fp.eval_last) {
        double rho, Yo[NK], T, f2[NK];
        errs |= state(NQ, rho, Yo, T, Tprev);
        production_pair(rho, T, Yo, f2);
        if (valid)
#pragma unroll
          for (int n = 0; n < NK; ++n)
            if (2 * n + sub < NS) F2(fp.F2new[NQ], 2 * n + sub)[i] = f2[n];
      }
      if (!valid) continue;
      if (errs) atomicOr(err, errs);
#pragma unroll
      for (int q = 0; q < 5; ++q)
        if ((q & 1) == sub) (Uo + q * nS)[s] = Un[q];
#pragma unroll
      for (int n = 0; n < NK; ++n)
        if (2 * n + sub < NS) (Uo + (5 + 2 * n + sub) * nS)[s] = Uk[n];
    }
  }
}

// The two kernels above fused for four coarse nodes, four fine sub-steps
// and at most nine species: the interval's increments are formed in registers with k_mr_src's
// arithmetic and consumed by k_mr_step's sub-steps without the round trip
// through HBM (4 nU stores and loads per cell).  The chemistry changes only
// the species components, so the other five follow from their increments
// alone: the prologue runs them through all sub-steps and keeps just the
// density and internal energy each temperature solve needs.  What stays live
// over the sub-steps (4 Ns species increments, Ns partial densities, 2 x 5
// scalars) fits the registers of the two waves per SIMD that the LDS column
// allows.  Sub-step r reads row 0 of each array, which then shifts up by one,
// so every register index is known at compile time.
template <int NS>
__global__ __launch_bounds__(256, 2) void k_mr_fused(const BoxDev *__restrict__ boxes,
                                                     const Item *__restrict__ items, int nitems,
                                                     TileShape ts, FRef Uin, FRef Uout,
                                                     const FineCoef *__restrict__ fc, FinePtrs fp,
                                                     const DevMech *__restrict__ m, int *err) {
  constexpr int NU = 5 + NS, NQ = 4, N1 = 4;
  NSDC_CHEM_LDS(NS, NSDC_CHEM_LDS_LIMIT, chem_sh);
  double *sh = chem_lds_setup<NS, NSDC_CHEM_LDS_LIMIT>(chem_sh, m);
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    int x, y, z;
    tile_cell(w, ts, x, y, z);
    if (x >= b.nx || y >= b.ny || z >= b.nz) continue;
    const long long nS = (long long)b.sx * b.sy * b.sz, nI = (long long)b.nx * b.ny * b.nz;
    const unsigned s = ((unsigned)(z + NSDC_NG) * b.sy + (y + NSDC_NG)) * b.sx + (x + NSDC_NG);
    const unsigned i = ((unsigned)z * b.ny + y) * b.nx + x;
    const long long o1 = b.offI * NU, o2 = b.offI * NS;
    auto F1 = [&](int slot, int q) { return fp.F1base + (slot * fp.f1slot + o1 + q * nI); };
    auto F2 = [&](int slot, int k) { return fp.F2base + (slot * fp.f2slot + o2 + k * nI); };
    const double dt = fp.dt;
    // the coefficients are read once per work item (hoisted out of the item
    // loop they would stay live, in more scalar registers than there are,
    // through the chemistry)
    asm volatile("" ::: "memory");
    double A[NQ][NU];
    // A[r][q], sub-step r, component q (k_mr_src's arithmetic; the S22 rows
    // padded with zeros to the interval's five fine nodes add exact zeros)
    auto increments = [&](int q) __attribute__((always_inline)) {
      double f1[N1];
#pragma unroll
      for (int j = 0; j < N1; ++j) f1[j] = F1(fp.F1old[j], q)[i];
      const double dF1 = F1(fp.F1new_p, q)[i] - F1(fp.F1old_p, q)[i];
      double g[NQ + 1];
      if (q >= 5) {
#pragma unroll
        for (int j = 0; j <= NQ; ++j) g[j] = F2(fp.F2old[j], q - 5)[i];
      }
#pragma unroll
      for (int r = 0; r < NQ; ++r) {
        const double dtq = fc->dtq[r] * dt;
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < N1; ++j) acc += fc->S21[r][j] * f1[j];
        double v = dtq * dF1 + dt * acc;
        if (q >= 5) {
          double s22 = 0.0;
#pragma unroll
          for (int j = 0; j <= NQ; ++j) s22 += fc->S22n[r][j] * g[j];
          v += dt * s22 - dtq * g[r];
        }
        A[r][q] = v;
      }
    };
    // the five non-species components first: their sub-step values are
    // formed before the species' increments take registers
#pragma unroll
    for (int q = 0; q < 5; ++q) increments(q);
    const double *Ui = Uin.get(w.box, b.offS * NU);
    double *Uo = Uout.get(w.box, b.offS * NU);
    // density and internal energy at sub-steps 0..NQ (as cell_state forms them)
    double Un[5], rq[NQ + 1], eq[NQ + 1];
#pragma unroll
    for (int c = 0; c < 5; ++c) Un[c] = (Ui + c * nS)[s];
#pragma unroll
    for (int r = 0; r <= NQ; ++r) {
      rq[r] = Un[0];
      const double ir = 1.0 / Un[0];
      const double ux = Un[1] * ir, uy = Un[2] * ir, uz = Un[3] * ir;
      eq[r] = Un[4] * ir - 0.5 * (ux * ux + uy * uy + uz * uz);
      if (r < NQ) {
#pragma unroll
        for (int c = 0; c < 5; ++c) Un[c] += A[r][c];
      }
    }
    // final values of the non-species components (each thread reads and
    // writes only its own cell, so the in-place case is safe)
#pragma unroll
    for (int c = 0; c < 5; ++c) (Uo + c * nS)[s] = Un[c];
#pragma unroll
    for (int q = 5; q < NU; ++q) increments(q);
    double Ys[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) Ys[k] = (Ui + (5 + k) * nS)[s];
    int errs = 0;
    double Tprev = 1000.0;
#pragma unroll 1
    for (int qq = 0; qq < NQ; ++qq) {
      double f2[NS];
      if (qq == 0 && fp.q0_known) {
#pragma unroll
        for (int k = 0; k < NS; ++k) f2[k] = F2(fp.F2old[0], k)[i];
      } else {
        double Y[NS], T;
        const double ir = 1.0 / rq[0];
#pragma unroll
        for (int k = 0; k < NS; ++k) Y[k] = Ys[k] * ir;
        errs |= rq[0] > 0.0 ? 0 : NSDC_ERR_RHO;
        errs |= temperature<NS>(m, Y, eq[0], T, Tprev);
        Tprev = T;
        production_any<NS, NSDC_CHEM_LDS_LIMIT>(m, rq[0], T, Y, f2, sh);
#pragma unroll
        for (int k = 0; k < NS; ++k) F2(fp.F2new[qq], k)[i] = f2[k];
      }
      const double dtq = fc->dtq[qq] * dt;
#pragma unroll
      for (int k = 0; k < NS; ++k) Ys[k] += A[0][5 + k] + dtq * f2[k];
#pragma unroll
      for (int r = 0; r + 1 < NQ; ++r)
#pragma unroll
        for (int k = 0; k < NS; ++k) A[r][5 + k] = A[r + 1][5 + k];
#pragma unroll
      for (int r = 0; r < NQ; ++r) {
        rq[r] = rq[r + 1];
        eq[r] = eq[r + 1];
      }
    }
    if (fp.eval_last) {
      double Y[NS], T, f2[NS];
      const double ir = 1.0 / rq[0];
#pragma unroll
      for (int k = 0; k < NS; ++k) Y[k] = Ys[k] * ir;
      errs |= rq[0] > 0.0 ? 0 : NSDC_ERR_RHO;
      errs |= temperature<NS>(m, Y, eq[0], T, Tprev);
      production_any<NS, NSDC_CHEM_LDS_LIMIT>(m, rq[0], T, Y, f2, sh);
#pragma unroll
      for (int k = 0; k < NS; ++k) F2(fp.F2new[NQ], k)[i] = f2[k];
    }
    if (errs) atomicOr(err, errs);
#pragma unroll
    for (int k = 0; k < NS; ++k) (Uo + (5 + k) * nS)[s] = Ys[k];
  }
}

}  // namespace nsdc

// ------------------------------------------------------------ launchers
#include "launch.h"

namespace nsdc {

// ------------------------------------------------ multirate SDC, mode 2
// Chemistry source w_k = W_k sum_j nu_kj q_j of the species densities y at
// fixed rho and internal energy, and the Newton matrix of the implicit solve
//   A = I - h dw/dy,
// dw/dy from mass action (dq_j/dc_m) and the Arrhenius and equilibrium
// temperature dependence (dq_j/dT) with the temperature following the
// species at fixed internal energy: dT/dy_m = -e_m(T) / (rho c_v).  The
// runtime-indexed per-cell arrays live in a slot sl (entry i at sl[i st]):
// in LDS (st = 64, one wave per workgroup, up to 9 species) or in the lane's
// slot of a workspace region (st = the launch's lanes):
//   A [NS][NS] | G [NS] | c [NS+1] | g [NS+1] | h/RT [NS+1] | aT [NS+1] | w [NS+1]
// (index NS of the last five is the dummy species of absent molecules); y
// and b stay in registers.
template <int NS>
struct Mr2Layout {
  static constexpr int A = 0, G = NS * NS, C = G + NS, GR = C + NS + 1, HR = GR + NS + 1, AT = HR + NS + 1,
                       W = AT + NS + 1;
};
static_assert(Mr2Layout<21>::W + 22 == NSDC_MR2_SLOT(21), "mode-2 slot layout");

// A slot in LDS: entry i at p[i st].  LANES lanes share it (add: LDS atomics
// for more than one).  ld/put take any index; ldv/putv are the same here.
template <int NS, int LANES>
struct Mr2SlotLds : Mr2Layout<NS> {
  double *p;
  int stride;
  __device__ double ld(int i) const { return p[i * stride]; }
  __device__ void put(int i, double v) const { p[i * stride] = v; }
  __device__ double ldv(int i) const { return ld(i); }
  __device__ void putv(int i, double v) const { put(i, v); }
  __device__ void add(int i, double v) const {
    if constexpr (LANES == 1)
      p[i * stride] += v;
    else
      atomicAdd(p + i * stride, v);
  }
};

// A lane's slot in a workspace region of NSDC_MR2_MAXWG * 256 lanes, entry i
// of lane l at byte 8 (i NSDC_MR2_MAXWG 256 + l), through a buffer resource:
// the lane's byte offset is its one vector offset and a wave-uniform index
// times the fixed stride rides in the scalar offset (with the index in a
// vector address every entry of an unrolled solve needed its own 64-bit
// address, which the compiler hoisted and spilled).  ldv/putv take a
// per-lane index (the pivot row) in the vector offset.
template <int NS>
struct Mr2SlotBuf : Mr2Layout<NS> {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  static constexpr int STRIDE = NSDC_MR2_MAXWG * 256 * 8;
  __amdgpu_buffer_rsrc_t r;
  int voff;
  __device__ double ld(int i) const {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, i * STRIDE, 0));
  }
  __device__ void put(int i, double v) const {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, i * STRIDE, 0);
  }
  __device__ double ldv(int i) const {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff + i * STRIDE, 0, 0));
  }
  __device__ void putv(int i, double v) const {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff + i * STRIDE, 0, 0);
  }
  __device__ void add(int i, double v) const { put(i, ld(i) + v); }
};
static_assert((long long)NSDC_MR2_SLOT(NSDC_NSMAX) * NSDC_MR2_MAXWG * 256 * 8 < (1LL << 31),
              "mode-2 workspace slots must stay within a buffer resource's signed offsets");

// LANES = 2: the two lanes of a cell (32 apart in one wave) share its slot
// in LDS; both write the same per-species values and form the same matrix
// (identical writes), each takes every other reaction and adds its terms
// with LDS atomics (a wave executes them in a fixed lane order).
template <int NS, int LANES, class Slot>
__device__ void mr2_rates_jacobian(const DevMech *__restrict__ m, const Slot &sl, const double *y,
                                   double rho, double T, double cv, double h, int sub = 0) {
  const double lnT = log(T), invT = 1.0 / T;
  // keep the mechanism's coefficient loads here: hoisted out of the Newton
  // iterations they outgrow the registers and are spilled and reloaded
  asm volatile("" ::: "memory");
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    sl.put(sl.C + k, y[k] * m->invW[k]);
    sl.put(sl.GR + k, g_RT(m, k, T, invT, lnT));
    sl.put(sl.HR + k, h_RT(m, k, T, invT));
    sl.put(sl.AT + k, 0.0);
    sl.put(sl.W + k, 0.0);
#pragma unroll
    for (int c = 0; c < NS; ++c) sl.put(sl.A + k * NS + c, 0.0);
  }
  sl.put(sl.C + NS, 1.0);
  sl.put(sl.GR + NS, 0.0);
  sl.put(sl.HR + NS, 0.0);
  sl.put(sl.AT + NS, 0.0);
  sl.put(sl.W + NS, 0.0);
  const double lnRTp = lnT + LN_RU_PREF;
  const int nr = m->nr;
  if constexpr (LANES > 1) wave_sync();
  for (int j = sub; j < nr; j += LANES) {
    const int sp[4] = {m->rs[j][0], m->rs[j][1], m->ps[j][0], m->ps[j][1]};
    const double lnkf = m->lnA[j] + m->beta[j] * lnT - m->EaR[j] * invT;
    const double dg = (sl.ld(sl.GR + sp[2]) + sl.ld(sl.GR + sp[3])) - (sl.ld(sl.GR + sp[0]) + sl.ld(sl.GR + sp[1]));
    const double kf = exp(lnkf);
    const double kr = exp(lnkf + dg + m->dnu[j] * lnRTp);
    const double c0 = sl.ld(sl.C + sp[0]), c1 = sl.ld(sl.C + sp[1]), c2 = sl.ld(sl.C + sp[2]),
                 c3 = sl.ld(sl.C + sp[3]);
    const double fwd = kf * c0 * c1, rev = kr * c2 * c3;
    const double q = fwd - rev;
    // d ln k_f / dT and d ln k_r / dT (d(g/RT)/dT = -(h/RT)/T)
    const double dlkf = (m->beta[j] + m->EaR[j] * invT) * invT;
    const double ddg =
        -((sl.ld(sl.HR + sp[2]) + sl.ld(sl.HR + sp[3])) - (sl.ld(sl.HR + sp[0]) + sl.ld(sl.HR + sp[1]))) * invT;
    const double dlkr = dlkf + ddg + m->dnu[j] * invT;
    const double dqdT = fwd * dlkf - rev * dlkr;
    // dq/dc of the four slots (a species twice gets both terms)
    const double dq[4] = {kf * c1, kf * c0, -kr * c3, -kr * c2};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double sgn = i < 2 ? -1.0 : 1.0;
      const int k = sp[i];
      sl.add(sl.W + k, sgn * q);
      sl.add(sl.AT + k, sgn * dqdT);
      if (k < NS)
#pragma unroll
        for (int l = 0; l < 4; ++l)
          if (sp[l] < NS) sl.add(sl.A + k * NS + sp[l], sgn * dq[l] * m->invW[sp[l]]);
    }
  }
  if constexpr (LANES > 1) wave_sync();
  // A = I - h W_k (d(sum nu q)/dy_m + aT_k dT/dy_m); w_k = W_k (sum nu q)_k
  const double irc = 1.0 / (rho * cv);
  double dTdy[NS];
#pragma unroll
  for (int c = 0; c < NS; ++c) dTdy[c] = -m->Rk[c] * T * (sl.ld(sl.HR + c) - 1.0) * irc;
  // (rows as a loop above twelve species, as in mr2_solve)
  constexpr int UROW = NS <= 12 ? NS : 1;
#pragma unroll UROW
  for (int k = 0; k < NS; ++k) {
    const double hW = h * m->W[k], aT = sl.ld(sl.AT + k);
#pragma unroll
    for (int c = 0; c < NS; ++c)
      sl.put(sl.A + k * NS + c, (k == c ? 1.0 : 0.0) - hW * (sl.ld(sl.A + k * NS + c) + aT * dTdy[c]));
    sl.put(sl.W + k, sl.ld(sl.W + k) * m->W[k]);
  }
}

// A x = G in place (x in G) by Gaussian elimination with partial pivoting.
template <int NS, class Slot>
__device__ void mr2_solve(const Slot &sl) {
  auto a = [&](int r, int c) { return sl.ld(sl.A + r * NS + c); };
  auto seta = [&](int r, int c, double v) { sl.put(sl.A + r * NS + c, v); };
  // unrolled up to twelve species; beyond, the unrolled elimination's
  // operands outgrow the registers (the 21-species kernel spilled 4.5 KB per
  // lane), so the column loop runs as a loop
  constexpr int UCOL = NS <= 12 ? NS : 1;
#pragma unroll UCOL
  for (int col = 0; col < NS; ++col) {
    int piv = col;
    double best = fabs(a(col, col));
#pragma unroll
    for (int r = col + 1; r < NS; ++r) {
      const double v = fabs(a(r, col));
      if (v > best) {
        best = v;
        piv = r;
      }
    }
    if (piv != col) {
      // (the pivot row differs between lanes: per-lane addressing)
#pragma unroll
      for (int c = col; c < NS; ++c) {
        const double t = a(col, c);
        seta(col, c, sl.ldv(sl.A + piv * NS + c));
        sl.putv(sl.A + piv * NS + c, t);
      }
      const double t = sl.ld(sl.G + col);
      sl.put(sl.G + col, sl.ldv(sl.G + piv));
      sl.putv(sl.G + piv, t);
    }
    const double inv = 1.0 / a(col, col);
#pragma unroll
    for (int r = col + 1; r < NS; ++r) {
      const double f = a(r, col) * inv;
#pragma unroll
      for (int c = col + 1; c < NS; ++c) seta(r, c, a(r, c) - f * a(col, c));
      sl.put(sl.G + r, sl.ld(sl.G + r) - f * sl.ld(sl.G + col));
    }
  }
#pragma unroll UCOL
  for (int r = NS - 1; r >= 0; --r) {
    double x = sl.ld(sl.G + r);
#pragma unroll
    for (int c = r + 1; c < NS; ++c) x -= a(r, c) * sl.ld(sl.G + c);
    sl.put(sl.G + r, x / a(r, r));
  }
}

// Implicit chemistry of one coarse interval (Mr2Imp): per cell the state
// U* = U_p + sum_j c1_j F1_j + sum_j c2_j F2_j - h F1_{p+1} (species part of
// the F1 terms only), then Newton's method on y - h w(y) = b for its species
// densities b (rho, rho u, rho E fixed, hence rho and the internal energy):
// stop one iteration after the first whose largest update is at most
// 1e-13 rho (at most 40; else NSDC_ERR_IMPLICIT).  Writes X = w(y*).
// LDS: up to 9 species, the slots in LDS, one wave per workgroup making as
// many passes over the interior tile as it has waves of cells; otherwise the
// workspace slots, one lane per cell of the tile.
template <int NS, bool LDS, int LANES = 1>
__global__ __launch_bounds__(LDS ? 64 : 256) void k_mr2_imp(const BoxDev *__restrict__ boxes,
                                                            const Item *__restrict__ items, int nitems,
                                                            TileShape ts, FRef Ucur, Mr2Imp a,
                                                            const DevMech *__restrict__ m, int *err) {
  constexpr int NU = 5 + NS;
  // LDS: CPP cells per pass, the LANES lanes of a cell CPP apart
  constexpr int CPP = 64 / LANES;
  static_assert(LANES == 1 || LDS, "lanes share a slot in LDS only");
  __shared__ double slot_sh[LDS ? NSDC_MR2_SLOT(NS) * CPP : 1];
  const int sub = LANES > 1 ? (int)threadIdx.x / CPP : 0, cslot = (int)threadIdx.x % CPP;
  // the slot: in LDS, or the lane's in the workspace region (at most
  // NSDC_MR2_MAXWG workgroups of at most 256 lanes)
  using Slot = std::conditional_t<LDS, Mr2SlotLds<NS, LANES>, Mr2SlotBuf<NS>>;
  Slot sl;
  if constexpr (LDS) {
    sl.p = slot_sh + cslot;
    sl.stride = CPP;
  } else {
    sl.r = __builtin_amdgcn_make_buffer_rsrc((void *)a.J, (short)0,
                                             (int)((long long)NSDC_MR2_SLOT(NS) * Mr2SlotBuf<NS>::STRIDE),
                                             0x00020000);
    sl.voff = (int)(blockIdx.x * blockDim.x + threadIdx.x) * 8;
  }
  const int tcells = ts.tx * ts.ty * ts.tz;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const Item w = items[it];
    const BoxDev b = boxes[w.box];
    for (int pass = 0; pass < (LDS ? (tcells + CPP - 1) / CPP : 1); ++pass) {
      int x, y, z;
      if constexpr (LDS) {
        const int lin = pass * CPP + cslot;
        if (lin >= tcells) continue;
        x = w.x0 + lin % ts.tx;
        y = w.y0 + (lin / ts.tx) % ts.ty;
        z = w.z0 + lin / (ts.tx * ts.ty);
      } else {
        tile_cell(w, ts, x, y, z);
      }
      if (x >= b.nx || y >= b.ny || z >= b.nz) continue;
      const long long nS = (long long)b.sx * b.sy * b.sz, nI = (long long)b.nx * b.ny * b.nz;
      const long long s = ((long long)(z + NSDC_NG) * b.sy + (y + NSDC_NG)) * b.sx + (x + NSDC_NG);
      const long long i = ((long long)z * b.ny + y) * b.nx + x;
      const long long o2 = b.offI * NU + i, o1 = b.offI * NS + i;
      const double *U = Ucur.get(w.box, b.offS * NU);
      double Us[5], yv[NS], bv[NS];
#pragma unroll
      for (int q = 0; q < NU; ++q) {
        double v = U[q * nS + s];
        for (int j = 0; j < a.n2; ++j) v += a.c2[j] * a.F2[j][o2 + q * nI];
        if (q >= 5) {
          for (int j = 0; j < a.n1; ++j) v += a.c1[j] * a.F1[j][o1 + (q - 5) * nI];
          v -= a.h * a.F1right[o1 + (q - 5) * nI];
          bv[q - 5] = v;
          yv[q - 5] = v;
        } else {
          Us[q] = v;
        }
      }
      const double rho = Us[0], ir = 1.0 / rho;
      const double e = Us[4] * ir - 0.5 * (Us[1] * Us[1] + Us[2] * Us[2] + Us[3] * Us[3]) * ir * ir;
      double T = 1000.0, Y[NS];
      int errs = rho > 0.0 ? 0 : NSDC_ERR_RHO;
      bool conv = false, done = false;
      for (int itn = 0; itn < 40 && !done; ++itn) {
#pragma unroll
        for (int k = 0; k < NS; ++k) Y[k] = yv[k] * ir;
        errs |= temperature<NS>(m, Y, e, T, T);
        double cv = 0.0;
#pragma unroll
        for (int k = 0; k < NS; ++k) cv += Y[k] * m->Rk[k] * (cp_R(m, k, T) - 1.0);
        mr2_rates_jacobian<NS, LANES>(m, sl, yv, rho, T, cv, a.h, sub);
#pragma unroll
        for (int k = 0; k < NS; ++k) sl.put(sl.G + k, yv[k] - a.h * sl.ld(sl.W + k) - bv[k]);
        mr2_solve<NS>(sl);
        double dmax = 0.0;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const double d = sl.ld(sl.G + k);
          yv[k] -= d;
          dmax = fmax(dmax, fabs(d));
        }
        done = conv;
        conv = !(dmax > 1e-13 * rho);   // (a NaN update never converges)
      }
      if (!done) errs |= NSDC_ERR_IMPLICIT;
#pragma unroll
      for (int k = 0; k < NS; ++k) Y[k] = yv[k] * ir;
      errs |= temperature<NS>(m, Y, e, T, T);
      double cv = 0.0;
#pragma unroll
      for (int k = 0; k < NS; ++k) cv += Y[k] * m->Rk[k] * (cp_R(m, k, T) - 1.0);
      mr2_rates_jacobian<NS, LANES>(m, sl, yv, rho, T, cv, a.h, sub);
#pragma unroll
      for (int k = 0; k < NS; ++k)
        if (LANES == 1 || k % LANES == sub) a.X[o1 + k * nI] = sl.ld(sl.W + k);
      if (errs) atomicOr(err, errs);
    }
  }
}

// Fine sub-step of eq. (mrupdate2) (Mr2Node).
template <int NS>
__global__ __launch_bounds__(256) void k_mr2_node(const BoxDev *__restrict__ boxes,
                                                  const Item *__restrict__ items, int nitems, TileShape ts,
                                                  FRef Ucur, FRef Unext, Mr2Node a) {
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
    const long long o2 = b.offI * NU + i, o1 = b.offI * NS + i;
    const double *Uc = Ucur.get(w.box, b.offS * NU);
    double *Un = Unext.get(w.box, b.offS * NU);
    for (int q = 0; q < NU; ++q) {
      const long long k2 = o2 + q * nI;
      double sq = 0.0;
      for (int j = 0; j < a.n2; ++j) sq += a.S22[j] * a.F2[j][k2];
      double corr = a.dtq * (a.F2new_q[k2] - a.F2old_q[k2]);
      if (q >= 5) {
        const long long k1 = o1 + (q - 5) * nI;
        for (int j = 0; j < a.n1; ++j) sq += a.S21[j] * a.F1[j][k1];
        corr += a.dtq * (a.X[k1] - a.F1right[k1]);
      }
      Un[q * nS + s] = Uc[q * nS + s] + corr + a.dt * sq;
    }
  }
}

// ------------------------------------------------ residual early exit
// Bookkeeping of the device-side decision (one thread): op 0 at the start of
// an sdc_step call (no residuals, no sweeps yet) and of its first step, op 1
// at the start of every later step, op 2 at the end of each step (the sweeps
// it took: those up to the one that ended it, else all K).
__global__ void k_resid_ctl(ResidCtl *ctl, int op, int K) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (op == 0) {
    ctl->count = 0;
    ctl->sweeps = 0;
  }
  if (op <= 1) {
    ctl->stop = 0;
    ctl->rprev = -1.0;
  }
  if (op == 2) ctl->sweeps += ctl->stop ? ctl->stop : K;
}

// After sweep k (from 0) of a step: |R^k| = max_c max|R_c| / max|U_0,c| from
// the reduced maxima out[0..2 nU) (components with a zero denominator left
// out), recorded; the step's sweeps end once it no longer shrinks by the
// ratio (or is exactly zero).
__global__ void k_resid_decide(ResidCtl *ctl, const double *__restrict__ out, int nU, double ratio, int k) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || ctl->stop) return;
  double r = 0.0;
  for (int q = 0; q < nU; ++q)
    if (out[nU + q] > 0.0) r = fmax(r, out[q] / out[nU + q]);
  if (ctl->count < NSDC_RESID_HIST) ctl->hist[ctl->count] = r;
  ctl->count += 1;
  if (r == 0.0 || (ctl->rprev >= 0.0 && ctl->rprev < ratio * r))
    ctl->stop = k + 1;
  else
    ctl->rprev = r;
}

// If sweep k ended the step: its end state (the sweep buffer Us, every box's
// nU stored fields at the box's offset) into the states the step returns
// (Ud, per box) and, when a next step recycles it, its f(U_M) into the array
// the last sweep's would occupy (n2 doubles; nothing when the two coincide).
__global__ __launch_bounds__(256) void k_resid_copy(const ResidCtl *__restrict__ ctl, int k,
                                                    const BoxDev *__restrict__ boxes, int nbox, int nU,
                                                    const double *__restrict__ Us, FRef Ud, const double *Fs,
                                                    double *Fd, long long n2) {
  if (ctl->stop != k + 1) return;
  const long long step = (long long)gridDim.x * blockDim.x, t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (int bx = 0; bx < nbox; ++bx) {
    const BoxDev b = boxes[bx];
    const long long off = b.offS * nU, n = (long long)b.sx * b.sy * b.sz * nU;
    const double *src = Us + off;
    double *dst = Ud.get(bx, off);
    for (long long i = t0; i < n; i += step) dst[i] = src[i];
  }
  if (Fs != Fd)
    for (long long i = t0; i < n2; i += step) Fd[i] = Fs[i];
}

void launch_resid_ctl(hipStream_t s, ResidCtl *ctl, int op, int K) {
  hipLaunchKernelGGL(k_resid_ctl, dim3(1), dim3(64), 0, s, ctl, op, K);
}
void launch_resid_decide(hipStream_t s, ResidCtl *ctl, const double *out, int nU, double ratio, int k) {
  hipLaunchKernelGGL(k_resid_decide, dim3(1), dim3(64), 0, s, ctl, out, nU, ratio, k);
}
void launch_resid_copy(hipStream_t s, const ResidCtl *ctl, int k, const BoxDev *boxes, int nbox, int nU,
                       const double *Us, FRef Ud, const double *Fs, double *Fd, long long n2) {
  hipLaunchKernelGGL(k_resid_copy, dim3(1024), dim3(256), 0, s, ctl, k, boxes, nbox, nU, Us, Ud, Fs, Fd, n2);
}

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
                       c.itemsG, c.nG, U, c.skip);
    prof_end(c.prof, K_GHOST, c.stream);
  }
  static void prims(const LaunchCtx &c, FRef U, double *P, FRef F, int out_mode, int warm, int store_x) {
    prof_begin(c.prof, K_PRIMS, c.stream);
    const dim3 grid(grid_for(c.nS, c.cap)), block(c.tsS.tx * c.tsS.ty * c.tsS.tz);
    if (out_mode == 2)
      hipLaunchKernelGGL((k_prims<NS, true>), grid, block, 0, c.stream, c.boxes, c.itemsS, c.nS, c.tsS, U, P, F,
                         out_mode, warm, store_x, c.mech, c.err, c.skip);
    else
      hipLaunchKernelGGL((k_prims<NS, false>), grid, block, 0, c.stream, c.boxes, c.itemsS, c.nS, c.tsS, U, P, F,
                         out_mode, warm, store_x, c.mech, c.err, c.skip);
    prof_end(c.prof, K_PRIMS, c.stream);
  }
  static void vgrad(const LaunchCtx &c, const double *P, double *G) {
    prof_begin(c.prof, K_VGRAD, c.stream);
    hipLaunchKernelGGL(k_vgrad<NS>, dim3(grid_for(c.nS, c.cap)), dim3(c.tsS.tx * c.tsS.ty * c.tsS.tz), 0,
                       c.stream, c.boxes, c.itemsS, c.nS, c.tsS, P, G, c.mech, c.skip);
    prof_end(c.prof, K_VGRAD, c.stream);
  }
  template <int D, bool FIXED, bool REF, bool WIDE>
  static void dir_k(const LaunchCtx &c, FRef U, const double *P, const double *G, FRef F, unsigned parts) {
    const TileShape ts = c.tsD[D];
    const dim3 grid(grid_for(c.nD[D], c.cap)), block(ts.tx * ts.ty * ts.tz);
    hipLaunchKernelGGL((k_dir<NS, D, FIXED, REF, WIDE, false>), grid, block, 0, c.stream, c.boxes, c.itemsD[D],
                       c.nD[D], ts, U, P, G, F, parts, c.mech, c.skip);
    // the boundary layers of boxes with physical boundaries along D (the
    // wide stencil is rejected with them)
    if constexpr (!WIDE) {
      if (c.nB[D] > 0) {
        const TileShape tb = c.tsB[D];
        hipLaunchKernelGGL((k_dir<NS, D, FIXED, REF, false, true>), dim3(grid_for(c.nB[D], c.cap)),
                           dim3(tb.tx * tb.ty * tb.tz), 0, c.stream, c.boxes, c.itemsB[D], c.nB[D], tb, U, P, G, F,
                           parts, c.mech, c.skip);
      }
    }
  }
  template <bool FIXED, bool REF, bool WIDE>
  static void dir_d(const LaunchCtx &c, int d, FRef U, const double *P, const double *G, FRef F, unsigned parts) {
    if (d == 0)
      dir_k<0, FIXED, REF, WIDE>(c, U, P, G, F, parts);
    else if (d == 1)
      dir_k<1, FIXED, REF, WIDE>(c, U, P, G, F, parts);
    else
      dir_k<2, FIXED, REF, WIDE>(c, U, P, G, F, parts);
  }
  static void dir(const LaunchCtx &c, int d, FRef U, const double *P, const double *G, FRef F,
                  unsigned parts) {
    const bool ref = c.ref_species >= 0;
    prof_begin(c.prof, K_DIR_X + d, c.stream);
    if (c.wide) {   // (the wide pairs do not use the narrow matrix)
      if (ref)
        dir_d<true, true, true>(c, d, U, P, G, F, parts);
      else
        dir_d<true, false, true>(c, d, U, P, G, F, parts);
    } else if (c.smc_stencil) {
      if (ref)
        dir_d<true, true, false>(c, d, U, P, G, F, parts);
      else
        dir_d<true, false, false>(c, d, U, P, G, F, parts);
    } else {
      if (ref)
        dir_d<false, true, false>(c, d, U, P, G, F, parts);
      else
        dir_d<false, false, false>(c, d, U, P, G, F, parts);
    }
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
                       c.stream, c.boxes, c.itemsI, c.nI, c.tsI, Ucur, Unext, a, c.skip);
    prof_end(c.prof, K_SDC_NODE, c.stream);
  }
  static void sdc_resid(const LaunchCtx &c, FRef U0, FRef UM, const ResidArgs &a) {
    const int nb = grid_for(c.nI, NSDC_RESID_BLOCKS);
    prof_begin(c.prof, K_SDC_RESID, c.stream);
    hipLaunchKernelGGL(k_sdc_resid<NS>, dim3(nb), dim3(c.tsI.tx * c.tsI.ty * c.tsI.tz), 0, c.stream, c.boxes,
                       c.itemsI, c.nI, c.tsI, U0, UM, a, c.skip);
    hipLaunchKernelGGL(k_rows_max, dim3(2 * (5 + NS)), dim3(256), 0, c.stream, a.partial, nb, 2 * (5 + NS), a.out,
                       c.skip);
    prof_end(c.prof, K_SDC_RESID, c.stream);
  }
  static void mr2_imp(const LaunchCtx &c, FRef Ucur, const Mr2Imp &a) {
    // the lanes' workspace slots bound the grid
    prof_begin(c.prof, K_MR2_IMP, c.stream);
    if constexpr (NS <= 9) {
      // the Newton matrices in LDS: one wave per workgroup
      hipLaunchKernelGGL((k_mr2_imp<NS, true>), dim3(grid_for(c.nI, c.cap)), dim3(64), 0, c.stream, c.boxes,
                         c.itemsI, c.nI, c.tsI, Ucur, a, c.mech, c.err);
    } else if constexpr (NS <= 12) {
      // two lanes per cell sharing its slot in LDS (one lane's slot would
      // leave one workgroup per compute unit)
      hipLaunchKernelGGL((k_mr2_imp<NS, true, 2>), dim3(grid_for(c.nI, c.cap)), dim3(64), 0, c.stream, c.boxes,
                         c.itemsI, c.nI, c.tsI, Ucur, a, c.mech, c.err);
    } else {
      // the lanes' workspace slots bound the grid (the workspace holds
      // NSDC_MR2_MAXWG workgroups of the interior tile)
      const int grid = grid_for(grid_for(c.nI, c.cap), NSDC_MR2_MAXWG), block = c.tsI.tx * c.tsI.ty * c.tsI.tz;
      Mr2Imp b = a;
      b.jstride = (long long)grid * block;
      hipLaunchKernelGGL((k_mr2_imp<NS, false>), dim3(grid), dim3(block), 0, c.stream, c.boxes, c.itemsI, c.nI,
                         c.tsI, Ucur, b, c.mech, c.err);
    }
    prof_end(c.prof, K_MR2_IMP, c.stream);
  }
  static void mr2_node(const LaunchCtx &c, FRef Ucur, FRef Unext, const Mr2Node &a) {
    prof_begin(c.prof, K_SDC_NODE, c.stream);
    hipLaunchKernelGGL(k_mr2_node<NS>, dim3(grid_for(c.nI, c.cap)), dim3(c.tsI.tx * c.tsI.ty * c.tsI.tz), 0,
                       c.stream, c.boxes, c.itemsI, c.nI, c.tsI, Ucur, Unext, a);
    prof_end(c.prof, K_SDC_NODE, c.stream);
  }
  static void mr_fine(const LaunchCtx &c, FRef Uin, FRef Uout, const FineCoef *fc,
                      const FinePtrs &fp, double *A, long long aslot) {
    const dim3 grid(grid_for(c.nI, c.cap)), block(c.tsI.tx * c.tsI.ty * c.tsI.tz);
    if constexpr (NS <= 9) {
      if (fp.nq == 4 && fp.n1 == 4 && c.fused_fine) {
        prof_begin(c.prof, K_MR_FINE, c.stream);
        hipLaunchKernelGGL(k_mr_fused<NS>, grid, block, 0, c.stream, c.boxes, c.itemsI, c.nI, c.tsI, Uin, Uout,
                           fc, fp, c.mech, c.err);
        prof_end(c.prof, K_MR_FINE, c.stream);
        return;
      }
    }
    if constexpr (NS > 9) {
      if (fp.nq == 4 && fp.n1 == 4 && c.fused_fine) {
        prof_begin(c.prof, K_MR_FINE, c.stream);
        hipLaunchKernelGGL(k_mr_pair_fused<NS>, grid, dim3(128), 0, c.stream, c.boxes, c.itemsI, c.nI, c.tsI,
                           Uin, Uout, fc, fp, c.mech, c.err);
        prof_end(c.prof, K_MR_FINE, c.stream);
        return;
      }
    }
    prof_begin(c.prof, K_MR_SRC, c.stream);
    if (fp.nq == 4)
      hipLaunchKernelGGL((k_mr_src<NS, 4>), grid, block, 0, c.stream, c.boxes, c.itemsI, c.nI, c.tsI, fc, fp, A,
                         aslot);
    else
      hipLaunchKernelGGL((k_mr_src<NS, 0>), grid, block, 0, c.stream, c.boxes, c.itemsI, c.nI, c.tsI, fc, fp, A,
                         aslot);
    prof_end(c.prof, K_MR_SRC, c.stream);
    prof_begin(c.prof, K_MR_FINE, c.stream);
    if constexpr (NS > 9)
      hipLaunchKernelGGL(k_mr_pair<NS>, grid, dim3(128), 0, c.stream, c.boxes, c.itemsI, c.nI, c.tsI, Uin, Uout, fc,
                         fp, A, aslot, c.mech, c.err);
    else
      hipLaunchKernelGGL(k_mr_step<NS>, grid, block, 0, c.stream, c.boxes, c.itemsI, c.nI, c.tsI, Uin, Uout, fc,
                         fp, A, aslot, c.mech, c.err);
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
  o.sdc_resid = &Launch<NS>::sdc_resid;
  o.mr_fine = &Launch<NS>::mr_fine;
  o.mr2_imp = &Launch<NS>::mr2_imp;
  o.mr2_node = &Launch<NS>::mr2_node;
  return o;
}
#define NSDC_OPS_DEF(n)                                                  \
  static_assert((n) >= 1 && (n) <= NSDC_NSMAX, "species count out of range"); \
  static const Ops OPS_##n = make_ops<n>();
NSDC_SPECIES_COUNTS(NSDC_OPS_DEF)
#undef NSDC_OPS_DEF

const Ops *ops_for(int ns) {
#define NSDC_OPS_CASE(n) \
  if (ns == (n)) return &OPS_##n;
  NSDC_SPECIES_COUNTS(NSDC_OPS_CASE)
#undef NSDC_OPS_CASE
  return nullptr;
}
}  // namespace nsdc
