// Internal layouts shared by the host driver and the device kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define NSDC_NG 4
#define NSDC_NSMAX 24

// Species counts the kernels are compiled for (each an instantiation of
// every kernel template, as a code generated for one mechanism would be);
// a build may pass its own list, e.g.
//   -D'NSDC_SPECIES_COUNTS(X)=X(9) X(15) X(21)'
// with every count in [1, NSDC_NSMAX].
#ifndef NSDC_SPECIES_COUNTS
#define NSDC_SPECIES_COUNTS(X) X(9) X(12) X(21)
#endif
#define NSDC_NRMAX 256
#define NSDC_MAXNODES 40
#define NSDC_MAXFINE 33

namespace nsdc {
// primitive fields stored per ghosted cell (their order: Layout, physics.h)
__host__ __device__ constexpr int prim_fields(int ns) { return 9 + 3 * ns; }
constexpr double RU = 8.31446261815324;               // J / (mol K)
constexpr double PREF = 101325.0;                     // Pa, the Gibbs energies' reference pressure
constexpr double LN_RU_PREF = -9.408091968943316;     // ln(RU / PREF)
}  // namespace nsdc

// device error word bits
#define NSDC_ERR_NEWTON 1
#define NSDC_ERR_TRANGE 2
#define NSDC_ERR_RHO 4
#define NSDC_ERR_IMPLICIT 8   // implicit chemistry (multirate mode 2): Newton did not converge

// Mechanism tables in device memory.  Thermodynamic polynomials are stored
// pre-scaled for Horner evaluation of c_p/R, h/(RT) and s/R; reactions as
// two reactant and two product species indices (ns = no molecule: a dummy
// species of unit concentration).
struct DevMech {
  int ns, nr;
  double Tlo, Thi;
  double mu_ref, inv_Tref, mu_exp, inv_Pr, bulk;
  double W[NSDC_NSMAX], invW[NSDC_NSMAX], Rk[NSDC_NSMAX], invLe[NSDC_NSMAX];
  double cp[NSDC_NSMAX][5];   // a1..a5
  double hc[NSDC_NSMAX][5];   // a1, a2/2, a3/3, a4/4, a5/5
  double h6[NSDC_NSMAX];      // a6
  double sc[NSDC_NSMAX][4];   // a2, a3/2, a4/3, a5/4
  double s7[NSDC_NSMAX];      // a7
  // g/(RT) = h/(RT) - s/R = gc0 - a1 ln T + T (gc1 + T (gc2 + T (gc3 + T gc4))) + a6 / T
  double gc[NSDC_NSMAX][5];   // a1 - a7, -a2/2, -a3/6, -a4/12, -a5/20
  double lnA[NSDC_NRMAX], beta[NSDC_NRMAX], EaR[NSDC_NRMAX];
  // ln k_f - G_r0 - G_r1 (G = g/RT, the dummy slot's G = -ln(R T / p_ref))
  // as one function of T: xc0 + xc1 ln T + xc2 / T + T (xc3 + T (xc4 + T
  // (xc5 + T xc6))); xc7 pads the row to 64 bytes
  double xc[NSDC_NRMAX][8];
  int rs[NSDC_NRMAX][2], ps[NSDC_NRMAX][2];
  int dnu[NSDC_NRMAX];
  double M[8][8];             // narrow-stencil matrix, [m+3][n+3]
  double B[9][9];             // face-difference matrix B_oc = M_{o-1,c-1} - M_{o,c}
  double e2tab[64];           // 2^(j/64), j = 0..63 (correctly rounded), for the rate exponentials
  int ref;                    // species diffusion: -1 correction velocity, k >= 0 reference species k
  // stencils near a physical boundary (Section 2.5), variant v = b + 4 high
  // for a cell b = 0..3 cells from the boundary below (high = 0) or above
  // (high = 1), on the nine samples centred on the cell: first-derivative
  // weights of the advective and the diffusive terms (times 1/h), and the
  // matrix of the second-derivative pairs, (a u_x)_x = sum_oc a_o K_oc u_c / h^2
  double bwA[8][9], bwD[8][9];
  double bK[8][9][9];
};

// One box of a batch.  offS / offI: offsets (in cells) of this box inside
// arena arrays laid out box after box with (stored | interior) cells per
// component.
struct BoxDev {
  int nx, ny, nz;
  int sx, sy, sz;
  int np;   // bit d: physical boundaries along d (the box_desc's nonperiodic)
  long long offS, offI;
  double idx[3], idx2[3];
};

// One work item: a tile origin of one box (interior or stored coordinates
// depending on the stage) or, for the ghost fill, a chunk of ghost cells.
struct Item {
  int box, x0, y0, z0;
};

// A field set: per-box pointer table (user arrays) or an arena base.
struct FRef {
  double *base;
  double *const *tab;
  __host__ __device__ double *get(int box, long long off) const {
    return tab ? tab[box] : base + off;
  }
};

struct TileShape {
  int tx, ty, tz;
};

// Single-rate SDC node update arguments (passed by value).
struct NodeArgs {
  const double *Fold[8];   // F^k at the nodes 0..M
  double S[8];             // row m of the node-to-node matrix S
  int nnodes;
  const double *Fnew_m, *Fold_m;
  double dtau, dt;
};

// SDC residual R = U_0 + dt q.F - U_M (eq. residual) of one step after a
// sweep: per component the largest |R| and the largest |U_0| over the
// interior cells, reduced to 2 nU values.  partial: [NSDC_RESID_BLOCKS][2 nU]
// per-workgroup maxima, out: [2 nU].
#define NSDC_RESID_BLOCKS 1024
struct ResidArgs {
  const double *F[8];   // F at the nodes 0..M (interior arrays)
  double q[8];          // last row of the integration matrix (normalised step)
  int nnodes;
  double dt;
  double *partial, *out;
};

// Device state of the residual early exit over one sdc_step call: stop is
// 0 while the current step sweeps, else the number of sweeps it took (the
// stage kernels of its remaining sweeps return at once); rprev the step's
// previous residual; count the residuals measured in the call (the first
// NSDC_RESID_HIST of them in hist); sweeps the sweeps the call performed.
#define NSDC_RESID_HIST 4096
struct ResidCtl {
  int stop, count, sweeps, pad;
  double rprev;
  double hist[NSDC_RESID_HIST];
};

// Coefficients of one coarse interval of the multirate sweep, in units of
// the step: rows of S_{2,1} and S_{2,2} restricted to the interval's fine
// nodes, and the fine sub-step lengths (device memory, one per interval).
struct FineCoef {
  double S21[NSDC_MAXFINE][8];
  double S22[NSDC_MAXFINE][9];   // row q over the nodes jlo[q] .. jlo[q] + nfine - 1 of its piece
  double S22n[4][5];   // four sub-steps: row q over all five fine nodes of the interval, zero outside its piece
  double dtq[NSDC_MAXFINE];
  int jlo[NSDC_MAXFINE];
  int n1;          // coarse nodes M1 + 1
  int nq;          // fine sub-steps in the interval
  int nfine;       // nodes of one fine polynomial piece
};

// Node arrays of one coarse interval (passed by value).  Node values live
// in two arenas (f1: nU components, f2: ns components) of equal-size slots;
// the roles of the slots change from sweep to sweep, so the kernel receives
// slot numbers rather than pointers.
struct FinePtrs {
  double *F1base, *F2base;             // arena bases
  long long f1slot, f2slot;            // doubles per slot
  unsigned short F1old[8];              // f1 at the coarse nodes, iteration k
  unsigned short F1new_p, F1old_p;      // f1 at the interval's left coarse node, k+1 and k
  unsigned short F2old[NSDC_MAXFINE];   // f2 at the interval's fine nodes, iteration k
  unsigned short F2new[NSDC_MAXFINE];   // f2 at the interval's fine nodes, iteration k+1
  int q0_known;    // f2 at the first fine node is the step-start value F2old[0]
  int eval_last;   // evaluate and store f2 at the interval's last fine node
  int nq;          // fine sub-steps of the interval (the same as the coefficient table's)
  int n1;          // coarse nodes (the same as the coefficient table's)
  double dt;
};

// Multirate SDC mode 2 (eq. mrupdate2): the chemistry f1 on the coarse nodes
// (ns components per cell), advection-diffusion f2 on the fine nodes (nU).
//
// Implicit solve of one coarse interval p: per cell, y - h w(y) = b for the
// species densities, b the species part of
//   U_p + sum_j c1_j F1_j + sum_j c2_j F2_j - h F1_{p+1}
// (c1, c2: dt times the interval's sums of S21 and S22 rows), h the coarse
// interval; the other components are those of the same sum.  X = w(y*).
// Above nine species each lane owns a slot of the workspace J (entry i at
// J[lane + i jstride], NSDC_MR2_SLOT(ns) entries) for its Newton matrix and
// runtime-indexed vectors; up to nine species they live in LDS.
#define NSDC_MR2_SLOT(ns) ((ns) * (ns) + 6 * (ns) + 5)
#define NSDC_MR2_MAXWG 512   // workgroups of the implicit kernel (the lane slots)
struct Mr2Imp {
  const double *F1[8];              // f1 at the coarse nodes, iteration k
  double c1[8];
  const double *F2[NSDC_MAXFINE];   // f2 at the interval's fine nodes, iteration k
  double c2[NSDC_MAXFINE];
  int n1, n2;
  const double *F1right;            // f1 at node p+1, iteration k
  double h;
  double *X;                        // out: f1 at node p+1, iteration k+1
  double *J;
  long long jstride;
};

// Fine sub-step q of eq. (mrupdate2):
//   U_{q+1} = U_q + dtq (X - F1_{p+1}) + dtq (F2new_q - F2old_q)
//             + dt (sum_j S22_qj F2old_j + sum_j S21_qj F1old_j)
struct Mr2Node {
  const double *F2[9];   // f2 (iteration k) at the nodes of sub-step q's fine piece
  double S22[9];
  int n2;
  const double *F1[8];   // f1 (iteration k) at the coarse nodes
  double S21[8];
  int n1;
  const double *F2new_q, *F2old_q, *X, *F1right;
  double dtq, dt;
};
