/* narrowsdc: right-hand side of the multicomponent reacting compressible
 * Navier-Stokes equations on periodic 3D boxes and its (multirate) spectral
 * deferred correction step, in FP64 on AMD Instinct MI355X (gfx950).
 *
 * Method: Emmett, Zhang & Bell, "High-order algorithms for compressible
 * reacting flow with complex chemistry" (arXiv 1309.7327).
 *   - state vector and equations: Section 2.1, eq. (cns)
 *   - eighth-order centred first derivative, eighth-order narrow stencil for
 *     d/dx(a du/dx): Section 2.2, eqs. (DaDu), (H) and the 8x8 matrix M
 *   - correction-velocity species fluxes with the chain rule: Section 2.1
 *     eqs. (fbar), (Vc) and Section 2.4
 *   - SDC sweep: Section 3.1, eq. (expsdc); MRSDC mode 1: Section 3.2,
 *     eq. (mrupdate)
 *   - adjoint forms: transposes of the operators above (vector-Jacobian
 *     products of the right-hand side and of the SDC step)
 *
 * Conventions for every entry point
 *   - Fields are FP64, component-major, x fastest: field[q][z][y][x].
 *     "Ghosted" arrays have NG = 4 ghost layers on every side (as the paper's
 *     q, D arrays of Listing 1), i.e. (nx+8)*(ny+8)*(nz+8) cells per
 *     component; "interior" arrays have nx*ny*nz cells per component.
 *   - State vector U = (rho, rho u, rho v, rho w, rho E, rho Y_1 .. rho Y_ns),
 *     nU = 5 + ns components, SI units.
 *   - All field pointers are device pointers owned by the caller, 8-byte
 *     aligned, not aliasing each other unless stated.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream) and returns after argument checks with one of the status codes
 *     below.  Failures detected on the device (temperature Newton solve not
 *     converged, temperature outside the polynomial range, non-positive
 *     density) set a per-context error word that last_status() returns.
 *   - A context is used from one host thread at a time.
 */
#ifndef NARROWSDC_H
#define NARROWSDC_H
#include <stddef.h>
#ifdef __cplusplus
extern "C" {
#endif

enum {
  SDC_OK = 0,
  SDC_EINVAL = -1,      /* bad argument (null pointer, size, unsupported ns) */
  SDC_ENOMECH = -2,     /* no mechanism set on the context */
  SDC_EHIP = -3,        /* HIP runtime error */
  SDC_ETEMP = -4,       /* device: temperature solve failed / out of range / rho <= 0 */
  SDC_ENOMEM = -5,      /* workspace too small or allocation failed */
};

/* parts of the right-hand side (rhs_eval): convective terms, diffusive
 * terms (viscous, conductive, species diffusion), chemistry source */
enum { RHS_HYP = 1, RHS_DIFF = 2, RHS_REACT = 4, RHS_AD = 3, RHS_ALL = 7 };

typedef struct sdc_context sdc_context;

/* One box.  nonperiodic: bit d (1 x, 2 y, 4 z) set for physical boundaries
 * at both ends of direction d instead of periodic wrap-around (Section 2.5):
 * the stencils along that direction drop in order near the boundary (the
 * fourth and third cells from it: sixth- and fourth-order centred first
 * derivatives and narrow stencils; the next cell: second-order centred
 * diffusion and third-order advection biased away from the boundary; the
 * boundary cell: one-sided second-order diffusion and third-order
 * advection), using interior cells only; the ghost layers along d are
 * filled with copies of the boundary cells and never read by a stencil.
 * Needs at least 8 cells along d and the narrow stencil; the adjoint covers
 * periodic boxes only (SDC_EINVAL).  The paper's characteristic boundary
 * conditions are not applied: the boundary cells evolve by the one-sided
 * stencils alone. */
typedef struct {
  int nx, ny, nz;     /* interior cells, each >= 1 */
  int ng;             /* ghost layers: must be 4 */
  double dx, dy, dz;  /* grid spacing, m */
  int nonperiodic;    /* 0: periodic in every direction */
} box_desc;

/* Chemical mechanism and transport model (host pointers, deep-copied by
 * set_mechanism).  Thermodynamics: single-range NASA-7 polynomials,
 * c_p/R = a1 + a2 T + a3 T^2 + a4 T^3 + a5 T^4, enthalpy constant a6,
 * entropy constant a7, valid on [Tlo, Thi].  Reactions: reversible,
 * k_f = A T^b exp(-Ea/(R T)), reverse constant from the equilibrium
 * constant of the NASA Gibbs energies at p_ref = 101325 Pa; at most two
 * reactant and two product molecules per reaction (coefficients 0..2).
 * Transport: mu = mu_ref (T/T_ref)^mu_exp, lambda = mu c_p / Pr,
 * rho D_k = lambda / (c_p Le_k), bulk viscosity xi = bulk_ratio * mu.
 * m47, m48: the two free parameters of the eighth-order narrow stencil. */
typedef struct {
  int ns, nr;            /* species (a count the library was built for, see
                            sdc_species_supported), reactions (<= 256) */
  const double *W;       /* [ns] molecular weights, kg/mol */
  const double *nasa;    /* [ns][7] */
  double Tlo, Thi;
  const double *A;       /* [nr] SI units of the forward order */
  const double *b;       /* [nr] */
  const double *Ea;      /* [nr] J/mol */
  const int *nu_f;       /* [nr][ns] reactant coefficients */
  const int *nu_r;       /* [nr][ns] product coefficients */
  const double *Le;      /* [ns] Lewis numbers */
  double mu_ref, T_ref, mu_exp, Pr, bulk_ratio;
  double m47, m48;
} mechanism_desc;

/* Time scheme.  n_fine == 0: single-rate SDC (eq. expsdc) on n_coarse
 * Gauss-Lobatto nodes with the full right-hand side.  n_fine >= 2: multirate
 * SDC with n_coarse Gauss-Lobatto coarse nodes and n_fine Gauss-Lobatto nodes
 * repeated fine_repeat times inside every coarse interval (fine_repeat = 1:
 * type (b); > 1: type (c)), in one of the two modes of Section 3.2:
 *   mode 1 (or 0): eq. (mrupdate), advection-diffusion on the coarse nodes,
 *     chemistry on the fine nodes, both explicit;
 *   mode 2: eq. (mrupdate2), the chemistry on the coarse nodes, implicit (in
 *     each coarse interval a backward-Euler solve of the chemistry, by
 *     Newton's method cell by cell, with the interval's explicit update as
 *     forcing gives f1 at the interval's right node), advection-diffusion on
 *     the fine nodes, explicit.  For stiff chemistry; a Newton solve that does
 *     not converge sets the device error word (SDC_ETEMP from last_status). */
typedef struct {
  int n_coarse;     /* 2..8 */
  int sweeps;       /* K >= 1 */
  int n_fine;       /* 0 or 2..9 */
  int fine_repeat;  /* >= 1 */
  int mode;         /* multirate mode: 0 or 1 (mode 1), 2 (mode 2) */
} sdc_scheme;

/* Create a context on HIP device `device`.  Owns the device copy of the
 * mechanism, scratch for rhs_eval (grown on demand with hipMalloc) and the
 * device error word. */
int sdc_context_create(sdc_context **out, int device);
int sdc_context_destroy(sdc_context *ctx);

/* Copy a mechanism to the device (synchronous).  Returns SDC_EINVAL for
 * unsupported sizes or reactions with more than two molecules per side. */
int set_mechanism(sdc_context *ctx, const mechanism_desc *mech);

/* 1 if the kernels were compiled for `ns` species, else 0 (no device call).
 * Every kernel is specialised for its species count, as a code generated
 * for one mechanism is; the default build covers 9, 12 and 21 species, and
 * the build's NSDC_SPECIES_COUNTS list (counts 1..24) sets others. */
int sdc_species_supported(int ns);

/* Conserved state from primitives on the interior: p, T [nz][ny][nx],
 * Y [ns][nz][ny][nx], u [3][nz][ny][nx] (device, interior layout) -> U
 * (device, ghosted; ghost layers filled periodically).  Ideal-gas mixture:
 * rho = p Wbar/(R T), rho E = rho (e(T, Y) + |u|^2/2) (Section 2.1). */
int prim_to_cons(sdc_context *ctx, const box_desc *box, const double *p, const double *T,
                 const double *Y, const double *u, double *U, void *stream);

/* Right-hand side dU/dt of eq. (cns) on the interior.
 * U: ghosted state; its ghost layers are overwritten by the periodic fill.
 * dUdt: interior, nU components, overwritten.  parts: RHS_* mask.
 * Uses context scratch (allocated on first use or growth). */
int rhs_eval(sdc_context *ctx, const box_desc *box, double *U, double *dUdt, unsigned parts,
             void *stream);

/* Size of the library's static scratch array (64 MiB), the device memory of
 * rhs_eval_static.  Each GPU the library runs on holds one copy of it until
 * the process ends. */
#define NSDC_STATIC_SCRATCH_BYTES (64u << 20)

/* rhs_eval for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels and results (bit for bit) as rhs_eval, but the work
 * list, primitives and velocity gradients live in the static scratch array
 * instead of context scratch, so the call makes no hipMalloc, hipFree or
 * other device or pinned allocation (the context's creation set up the
 * array's address and a pinned staging buffer for the work list, which the
 * call copies to the device on `stream`).
 * Limit: the box's scratch (work list, (18 + 3 ns) doubles per ghosted
 * cell) must fit NSDC_STATIC_SCRATCH_BYTES, e.g. a 48^3 box with 9 species
 * or a 32^3 box with 21; larger boxes return SDC_EINVAL (use rhs_eval).
 * Every call on one GPU shares that GPU's array and it keeps the last call's
 * contents: calls that overlap on one GPU (other streams, other contexts,
 * other threads) race and must be ordered by the caller.  The profiler
 * (sdc_profile_enable) does not time these launches.  SDC_EHIP if the array's
 * address could not be obtained at context creation. */
int rhs_eval_static(sdc_context *ctx, const box_desc *box, double *U, double *dUdt, unsigned parts,
                    void *stream);

/* Bytes of device workspace sdc_step / sdc_step_batched need. */
int sdc_workspace_size(const sdc_context *ctx, int nbox, const box_desc *boxes,
                       const sdc_scheme *scheme, size_t *bytes);

/* Advance U (ghosted, in place) by nsteps steps of size dt with the scheme.
 * f(U_0) is recycled across the steps of one call.  workspace: caller-owned
 * device memory of at least sdc_workspace_size bytes holding every field
 * array of the step.  The first call for a box (and for a multirate scheme)
 * allocates the context's small work-list and coefficient tables; later
 * calls with the same box and scheme allocate nothing. */
int sdc_step(sdc_context *ctx, const box_desc *box, double *U, double dt, int nsteps,
             const sdc_scheme *scheme, void *workspace, size_t ws_bytes, void *stream);

/* Same for nbox independent periodic boxes advanced together: every stage
 * is one launch over a (box, tile) work list covering all boxes.
 * U[i] is box i's ghosted state (device pointer, host array of pointers). */
int sdc_step_batched(sdc_context *ctx, int nbox, const box_desc *boxes, double *const *U,
                     double dt, int nsteps, const sdc_scheme *scheme, void *workspace,
                     size_t ws_bytes, void *stream);

/* Second derivatives (a u_x)_x of the viscous, conduction and diffusion
 * terms (Section 2.2): enable = 0 (default) the eighth-order narrow stencil
 * of eq. (H); enable != 0 the wide stencil D(a D u), two applications of the
 * eighth-order first derivative, whose samples reach 8 cells (taken from the
 * periodic images).  The wide operator is blind to the grid's odd-even
 * mode, the reason the paper prefers the narrow one.  rhs_vjp and
 * sdc_step_vjp return SDC_EINVAL while it is on. */
int set_wide_stencil(sdc_context *ctx, int enable);

/* Kernel choice for the fine sub-steps of a multirate sweep (eq. mrupdate),
 * a tuning switch that leaves results unchanged bit for bit: enable != 0
 * (default) runs them as one kernel per coarse interval wherever the scheme
 * has four coarse nodes and four fine sub-steps per interval (the quadrature
 * increments stay on chip; above nine species the two lanes of a cell split
 * them by species); enable = 0, and every other case, uses a streaming
 * quadrature kernel followed by the sub-step kernel. */
int sdc_set_fused_fine(sdc_context *ctx, int enable);

/* SDC residual early exit (the residual of eq. residual, R^k = U_0 +
 * dt q.F^k - U_M^k, q the last row of the integration matrix): ratio = 0
 * (default) runs every step's K sweeps; ratio > 1 measures |R^k| after every
 * sweep but a step's last and skips the step's remaining sweeps once
 * |R^{k-1}| / |R^k| < ratio (the sweeps no longer approach the collocation
 * solution).  |R| is the largest over state components of max|R_c| /
 * max|U_0,c| over the interior; for sdc_step_batched both maxima run over
 * every box of the batch, whose boxes share the decision.  The decision is
 * taken on the device (the stage kernels of a step's skipped sweeps are
 * launched and return at once), so the call does not synchronise the stream
 * and may be captured in a graph like any other.  Covers single-rate
 * schemes: multirate schemes return SDC_EINVAL while it is on, and so do
 * rhs_vjp and sdc_step_vjp.  Enabling it allocates a small device buffer (kept until the
 * context is destroyed).  Errors: SDC_EINVAL for 0 < ratio <= 1 or ratio < 0. */
int sdc_set_residual_exit(sdc_context *ctx, double ratio);

/* The residuals |R^k| measured by the last sdc_step or sdc_step_batched call, in order (the
 * first max of them into norms, host memory), how many there were
 * (count, at most 4096 are kept) and the sweeps the call performed over all
 * its steps (sweeps); count and sweeps may be null.  After a call with the
 * residual early exit it synchronises the device (the decisions are in
 * device memory). */
int sdc_residual_history(const sdc_context *ctx, int max, double *norms, int *count, int *sweeps);

/* Graph mode (enable != 0): sdc_step / sdc_step_batched on a non-null stream
 * capture all launches of a call into a HIP graph the first time and replay
 * it for calls with identical arguments (same boxes, state pointers, dt,
 * nsteps, scheme and workspace).  Capture allocates the graph; replays
 * allocate nothing.  Disabling frees the cached graphs. */
int sdc_set_graph(sdc_context *ctx, int enable);

/* Tile-shape autotuner for a box set: times one full right-hand-side
 * evaluation over all boxes for each candidate workgroup tile shape and
 * persistent-grid size, and keeps the fastest for later calls on boxes of
 * these dimensions.  U[i]: the boxes' ghosted states (device; ghosts are
 * refilled, interiors untouched).  workspace: device scratch of at least
 * the sdc_workspace_size of a single-rate scheme for these boxes.  choice
 * (may be null) receives tile x, y, z and the workgroup cap (0 = one
 * workgroup per tile).  Results do not depend on the choice. */
int sdc_autotune(sdc_context *ctx, int nbox, const box_desc *boxes, double *const *U,
                 void *workspace, size_t ws_bytes, void *stream, int *choice);

/* ---- adjoint forms ----------------------------------------------------
 * Vector-Jacobian product of rhs_eval (the transpose of eq. cns as
 * discretised in Section 2.2, stage by stage: stencils, conserved ->
 * primitive map with the implicit-function derivative of the Newton
 * temperature, chemistry source):
 *   U_bar   += (d rhs / dU)^T dUdt_bar          (interior, nU components)
 *   lnA_bar += (d rhs / d ln A_j)^T dUdt_bar     (device [nr]; may be null)
 * U: ghosted state (device); its ghost layers are overwritten by the
 * periodic fill, its interior is read only.  dUdt_bar: interior cotangent
 * (device).  parts: RHS_* mask as in rhs_eval.  Uses context scratch
 * (allocated on first use or growth).  Both outputs are accumulated, in a
 * fixed order (no atomics): repeated calls give identical results. */
int rhs_vjp(sdc_context *ctx, const box_desc *box, double *U, const double *dUdt_bar,
            double *U_bar, double *lnA_bar, unsigned parts, void *stream);

/* Replace ln A_j of every reaction of the current mechanism (host array
 * [nr], synchronous).  Lets callers differentiate with respect to the
 * pre-exponential factors at values of their choice. */
int set_log_prefactors(sdc_context *ctx, const double *lnA);

/* Species diffusion consistent with mass conservation (Section 2.1).
 * k = -1 (the default after set_mechanism): correction velocity V_c, the
 * chain-rule form of Section 2.4.  k in [0, ns): reference species k, e.g.
 * N2: species j != k carry the mixture-model flux Fbar_j, species k carries
 * -sum_{j != k} Fbar_j, and the energy flux is sum_{j != k} Fbar_j (h_j -
 * h_k) (Section 2.4); no correction velocity.  Synchronous (waits for the
 * device before updating its copy of the mechanism).  Errors: SDC_ENOMECH
 * without a mechanism, SDC_EINVAL for k outside [-1, ns).  rhs_vjp and
 * sdc_step_vjp return SDC_EINVAL while a reference species is set. */
int set_reference_species(sdc_context *ctx, int k);

/* Bytes of device workspace sdc_step_vjp needs for nsteps steps. */
int sdc_vjp_workspace_size(const sdc_context *ctx, const box_desc *box, const sdc_scheme *scheme,
                           int nsteps, size_t *bytes);

/* Adjoint of nsteps single-rate SDC steps (eq. expsdc; n_fine must be 0)
 * of size dt from the state U0 (ghosted; ghost layers overwritten, interior
 * unchanged):
 *   U0_bar   = (d U_N / d U_0)^T UN_bar         (interior, overwritten)
 *   lnA_bar += (d U_N / d ln A)^T UN_bar        (device [nr]; may be null)
 * The forward steps are re-run to store the step-start states in the
 * workspace; each step's node states are then recomputed from its
 * checkpoint and swept backwards (one rhs_vjp per stored right-hand side).
 * workspace: caller-owned device memory of sdc_vjp_workspace_size bytes. */
int sdc_step_vjp(sdc_context *ctx, const box_desc *box, double *U0, double dt, int nsteps,
                 const sdc_scheme *scheme, const double *UN_bar, double *U0_bar, double *lnA_bar,
                 void *workspace, size_t ws_bytes, void *stream);

/* Synchronise `stream`, return and clear the device error word (SDC_OK or
 * SDC_ETEMP). */
int last_status(sdc_context *ctx, void *stream);

/* Text of the last error returned by a call on this context. */
const char *last_error_message(const sdc_context *ctx);

/* ---- measurement and tuning hooks ------------------------------------
 * sdc_profile_enable: attach (1, clearing previous records) or detach (0)
 *   per-kernel timers; while attached every launch is bracketed by HIP
 *   events recorded on its own stream.
 * sdc_profile_read: synchronise `stream`, write the summed duration (ms)
 *   and launch count of every kernel kind into total_ms[], count[] (arrays of
 *   at least 32 entries), clear the records; returns the number of kinds.
 * sdc_kernel_name: name of kernel kind `id` ("" if out of range).
 * sdc_set_tiles: force the tile shapes (threads x, y, z; product <= 256,
 *   interior product a multiple of 64) of the interior and stored index
 *   spaces, each independently (all three extents 0 = automatic) and cap
 *   the number of workgroups per launch (0 = one per work item); an extent
 *   set that mixes zero and non-zero values, a negative value or a
 *   negative cap returns SDC_EINVAL.  Forcing either shape bypasses the
 *   autotuner's choice for later plans. */
int sdc_profile_enable(sdc_context *ctx, int enable);
int sdc_profile_read(sdc_context *ctx, void *stream, double *total_ms, int *count);
const char *sdc_kernel_name(int id);
int sdc_set_tiles(sdc_context *ctx, int ix, int iy, int iz, int sx, int sy, int sz, int grid_cap);

#ifdef __cplusplus
}
#endif
#endif
