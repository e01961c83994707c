// Host-side interface to the adjoint (vector-Jacobian product) kernels.
#pragma once
#include "launch.h"

namespace nsdc {

// Adjoint accumulators on the stored (ghosted) cells of the boxes, laid out
// like the state (Ub, 5 + ns fields), the primitive fields (Pb) and the
// velocity gradient (Gb, 9 fields).
struct AdjBufs {
  double *Ub, *Pb, *Gb;
};

constexpr int ADJ_MAXT = 10;
struct AxpyArgs {
  double *Y[ADJ_MAXT];
  double c[ADJ_MAXT];
  int nt;
};
struct LincombArgs {
  const double *X[ADJ_MAXT];
  double c[ADJ_MAXT];
  int nt;
};

struct AdjOps {
  int ns;
  // transpose of the direction-d terms (coef: per-cell scratch, 7 interior
  // fields)
  void (*dir)(const LaunchCtx &, int d, const double *U, const double *P, const double *G, const double *V,
              const AdjBufs &, double *coef, unsigned parts);
  // returns the number of workgroups (rows of `partial`)
  int (*chem)(const LaunchCtx &, const double *U, const double *V, const AdjBufs &, double *partial);
  void (*vgrad)(const LaunchCtx &, const AdjBufs &);
  void (*prims)(const LaunchCtx &, const double *U, const AdjBufs &);
  void (*fold)(const LaunchCtx &, const AdjBufs &, double *out);
};

const AdjOps *adj_ops_for(int ns);
void adj_fill0(const LaunchCtx &c, double *p, long long n);
void adj_axpy(const LaunchCtx &c, const double *X, const AxpyArgs &a, long long n);
void adj_lincomb(const LaunchCtx &c, const LincombArgs &a, double *Y, long long n);
void adj_lnA_reduce(const LaunchCtx &c, const double *partial, int nblocks, int nr, double *lnA_bar);

}  // namespace nsdc
