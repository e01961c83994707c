// Host-side interface to the kernels: one table of launch functions per
// supported species count.
#pragma once
#include "nsdc_internal.h"

namespace nsdc {


// Kernel identities for the per-kernel timers.
enum KernelId {
  K_PRIM_TO_CONS = 0, K_GHOST, K_PRIMS, K_VGRAD, K_DIR_X, K_DIR_Y, K_DIR_Z, K_CHEM, K_SDC_NODE,
  K_MR_FINE, K_MR_SRC, K_DIR_ADJ_X, K_DIR_ADJ_Y, K_DIR_ADJ_Z, K_CHEM_ADJ, K_VGRAD_ADJ, K_PRIMS_ADJ,
  K_FOLD, K_ADJ_LINALG, K_SDC_RESID, K_MR2_IMP, K_NKERNELS
};
struct Profiler;
// Record a HIP event on `s` before (begin) / after (end) a launch of kernel `id`
// when a profiler is attached (no-ops otherwise).
void prof_begin(Profiler *p, int id, hipStream_t s);
void prof_end(Profiler *p, int id, hipStream_t s);

// Everything a launch needs besides its field pointers: the box table, the
// work-item lists of the three index spaces (interior tiles, stored tiles,
// ghost-cell chunks), their tile shapes and the grid-size cap.  Lists are
// stored in XCD order: workgroups are dispatched round-robin over the eight
// XCDs, and the list is permuted so that the workgroups of one XCD take a
// contiguous run of tiles in each round (neighbouring tiles share its L2).
struct LaunchCtx {
  hipStream_t stream;
  const BoxDev *boxes;
  const Item *itemsI, *itemsS, *itemsG;
  const Item *itemsD[3];   // interior lists of the stencil passes, direction D fastest
  int nD[3];
  TileShape tsD[3];
  const Item *itemsB[3];   // boundary layers of the directions with physical boundaries
  int nB[3];
  TileShape tsB[3];
  int nI, nS, nG;
  TileShape tsI, tsS;
  int cap;
  const DevMech *mech;
  int *err;
  Profiler *prof;
  bool smc_stencil;   // the default narrow-stencil parameters: compile-time B
  int ref_species;    // species diffusion: -1 correction velocity, else the reference species
  bool wide;          // second-derivative pairs with the wide stencil D(a D u)
  bool fused_fine;    // multirate fine sub-steps in one kernel where it applies
  // device flag of the residual early exit (null: none): non-zero once a
  // step's sweeps have ended, the stage kernels of the rest of the step
  // return at once
  const int *skip;
};

struct Ops {
  int ns;
  void (*prim_to_cons)(const LaunchCtx &, const double *, const double *, const double *,
                       const double *, FRef);
  void (*ghost)(const LaunchCtx &, FRef);
  // store_x = 0: leave the mole-fraction and species-enthalpy fields of P
  // unwritten (no pass of the evaluation reads them)
  void (*prims)(const LaunchCtx &, FRef, double *, FRef, int out_mode, int warm, int store_x);
  void (*vgrad)(const LaunchCtx &, const double *, double *);
  void (*dir)(const LaunchCtx &, int, FRef, const double *, const double *, FRef, unsigned);
  void (*chem)(const LaunchCtx &, FRef, double *);
  void (*sdc_node)(const LaunchCtx &, FRef, FRef, const NodeArgs &);
  void (*sdc_resid)(const LaunchCtx &, FRef U0, FRef UM, const ResidArgs &);
  void (*mr_fine)(const LaunchCtx &, FRef, FRef, const FineCoef *, const FinePtrs &, double *, long long);
  void (*mr2_imp)(const LaunchCtx &, FRef, const Mr2Imp &);
  void (*mr2_node)(const LaunchCtx &, FRef, FRef, const Mr2Node &);
};

// residual early exit decided on the device (kernels.hip)
void launch_resid_ctl(hipStream_t s, ResidCtl *ctl, int op, int K);
void launch_resid_decide(hipStream_t s, ResidCtl *ctl, const double *out, int nU, double ratio, int k);
void launch_resid_copy(hipStream_t s, const ResidCtl *ctl, int k, const BoxDev *boxes, int nbox, int nU,
                       const double *Us, FRef Ud, const double *Fs, double *Fd, long long n2);

// nullptr for an unsupported species count
const Ops *ops_for(int ns);

}  // namespace nsdc
