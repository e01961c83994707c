/* Oracle: plain, slow CPU FP64 reference for the reacting Navier-Stokes
 * right-hand side and its building blocks.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls
 * this code; only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, headers or tables with the HIP path.
 *
 * Conventions: fields are [component][z][y][x] with x fastest.  Interior
 * arrays have nx*ny*nz cells per component; the oracle builds its own
 * 4-layer periodic ghost copy internally.
 *
 * Return codes: 0 ok, -1 bad argument, -4 temperature solve failed or
 * temperature outside the polynomial fit range.
 */
#ifndef ORACLE_H
#define ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int ns, nr;
  const double *W;    /* [ns] kg/mol */
  const double *nasa; /* [ns][7]: c_p/R = a1+a2T+a3T^2+a4T^3+a5T^4, a6 enthalpy, a7 entropy constants */
  double Tlo, Thi;
  const double *A, *b, *Ea; /* [nr] SI, -, J/mol */
  const int *nu_f, *nu_r;   /* [nr][ns] */
  const double *Le;         /* [ns] Lewis numbers */
  double mu_ref, T_ref, mu_exp, Pr, bulk_ratio;
  double m47, m48;
  /* species diffusion consistent with mass conservation (Section 2.1): -1
     correction velocity; k >= 0 reference species k, whose flux is minus the
     sum of the others' mixture-model fluxes */
  int ref_species;
  /* second derivatives (a u_x)_x: 0 the narrow stencil (eq. H), 1 the wide
     stencil D(a D u) of two eighth-order first derivatives (Section 2.2) */
  int wide_stencil;
  /* bit d set: direction d has physical (non-periodic) boundaries at both
     ends, with the reduced-order boundary stencils of Section 2.5 (needs at
     least 8 interior cells along d and the narrow stencil) */
  int nonperiodic;
} omech;

enum { ORC_HYP = 1, ORC_DIFF = 2, ORC_REACT = 4 };

/* 8x8 narrow-stencil matrix of the paper's eighth-order family (Section 2.2),
 * row-major, entry [(m+3)*8 + (n+3)] for offsets m, n in -3..4. */
void oracle_narrow_matrix(double m47, double m48, double *M);
/* 6x6 matrix of the sixth-order family, entry [(m+2)*6 + (n+2)], m,n in -2..3. */
void oracle_narrow6_matrix(double m36, double *M);

/* Operators at the centre of a 9-sample line f[0..8] (index 4 = centre). */
double oracle_d1_point(const double *f9, double dx);
double oracle_narrow_point(const double *a9, const double *u9, double dx, double m47, double m48);

/* A line of n >= 8 points with physical boundaries at both ends: the first
 * derivative (kind 0 advection, 1 diffusion) and d/dx(a du/dx) with the
 * boundary stencils of Section 2.5 (eighth-order stencils from the fifth
 * point on). */
void oracle_d1_line(int n, const double *f, double dx, int kind, double *out);
void oracle_narrow_line(int n, const double *a, const double *u, double dx, double m47, double m48,
                        double *out);
/* 4x4 matrix of the fourth-order narrow stencil, entry [(m+1)*4 + (n+1)], m,n in -1..2. */
void oracle_narrow4_matrix(double *M);

/* Periodic 1D and 2D operators. */
void oracle_d1_periodic(int n, const double *f, double dx, double *out);
void oracle_narrow_periodic(int n, const double *a, const double *u, double dx, double m47,
                            double m48, double *out);
/* (a u_x)_x + (b u_y)_y on an n x n periodic grid, arrays [y][x]. */
void oracle_heat2d(int n, const double *a, const double *b, const double *u, double dx,
                   double m47, double m48, double *out);

/* Pointwise thermochemistry. */
void oracle_species_thermo(const omech *m, double T, double *cp_R, double *h_RT, double *s_R);
/* forward and reverse rate constants (SI) of every reaction at temperature T */
void oracle_rate_constants(const omech *m, double T, double *kf, double *kr);
int oracle_prim_to_cons(const omech *m, long ncell, const double *p, const double *T,
                        const double *Y, const double *u, double *U);
/* primitive fields from conserved: out [rho,u,v,w,T,p] (6 x ncell) */
int oracle_cons_to_prim(const omech *m, long ncell, const double *U, double *out);
/* speed of sound sqrt(gamma p / rho) of every cell */
int oracle_sound_speed(const omech *m, long ncell, const double *U, double *c);
/* rho*omega_k for every cell: out [ns][ncell] */
int oracle_production(const omech *m, long ncell, const double *U, double *wdot);

/* Full right-hand side on the interior of a periodic box.  parts is a mask of
 * ORC_HYP (convective), ORC_DIFF (viscous, conductive, species diffusion with
 * correction velocity) and ORC_REACT (chemistry source). */
int oracle_rhs(const omech *m, int nx, int ny, int nz, double dx, double dy, double dz,
               const double *U, unsigned parts, double *out, int nthreads);
/* Same, only at listed interior cells (cells[3*i] = x, y, z); out [ncells][nU]. */
int oracle_rhs_cells(const omech *m, int nx, int ny, int nz, double dx, double dy, double dz,
                     const double *U, unsigned parts, int ncells, const int *cells, double *out,
                     int nthreads);
/* Jacobian-vector product by forward-mode dual numbers: out = d rhs / dU . wU
 * + d rhs / d lnA . wA (wA may be null). */
int oracle_rhs_jvp(const omech *m, int nx, int ny, int nz, double dx, double dy, double dz,
                   const double *U, const double *wU, const double *wA, unsigned parts,
                   double *out, double *jvp, int nthreads);
/* The same product evaluated only at listed interior cells (cells[3*i] = x,
 * y, z); jvp [ncells][nU]. */
int oracle_rhs_jvp_cells(const omech *m, int nx, int ny, int nz, double dx, double dy, double dz,
                         const double *U, const double *wU, const double *wA, unsigned parts,
                         int ncells, const int *cells, double *jvp, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
