// Test driver: runs the oracle's entry points under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_oracle_sanitized.py with
// g++ -fsanitize=address,undefined, CPU only).  Reads one case from a raw
// binary file and writes the results for comparison with the regular build.
//
// Input layout: int32[8] = ns, nr, nx, ny, nz, ref_species, wide, 0;
// doubles W[ns], nasa[7 ns], A[nr], b[nr], Ea[nr], Le[ns], then Tlo, Thi,
// mu_ref, T_ref, mu_exp, Pr, bulk_ratio, m47, m48, dx; int32 nu_f[nr ns],
// nu_r[nr ns]; doubles U[nU n], wU[nU n], wA[nr] (n = nx ny nz).
// Output: doubles rhs[nU n], jvp[nU n], production[ns n], cells[4][nU].
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../oracle/oracle.h"

template <class T>
static void rd(FILE *f, T *p, size_t n) {
  if (fread(p, sizeof(T), n, f) != n) {
    fprintf(stderr, "short read\n");
    exit(2);
  }
}

int main(int argc, char **argv) {
  if (argc != 3) return 2;
  FILE *f = fopen(argv[1], "rb");
  if (!f) return 2;
  int hd[8];
  rd(f, hd, 8);
  const int ns = hd[0], nr = hd[1], nx = hd[2], ny = hd[3], nz = hd[4];
  const long n = (long)nx * ny * nz;
  const int nU = 5 + ns;
  std::vector<double> W(ns), nasa(7 * ns), A(nr), b(nr), Ea(nr), Le(ns), sc(10);
  rd(f, W.data(), ns);
  rd(f, nasa.data(), 7 * ns);
  rd(f, A.data(), nr);
  rd(f, b.data(), nr);
  rd(f, Ea.data(), nr);
  rd(f, Le.data(), ns);
  rd(f, sc.data(), 10);
  std::vector<int> nuf(nr * ns), nur(nr * ns);
  rd(f, nuf.data(), nuf.size());
  rd(f, nur.data(), nur.size());
  std::vector<double> U(nU * n), wU(nU * n), wA(nr);
  rd(f, U.data(), U.size());
  rd(f, wU.data(), wU.size());
  rd(f, wA.data(), nr);
  fclose(f);
  omech m{};
  m.ns = ns;
  m.nr = nr;
  m.W = W.data();
  m.nasa = nasa.data();
  m.Tlo = sc[0];
  m.Thi = sc[1];
  m.A = A.data();
  m.b = b.data();
  m.Ea = Ea.data();
  m.nu_f = nuf.data();
  m.nu_r = nur.data();
  m.Le = Le.data();
  m.mu_ref = sc[2];
  m.T_ref = sc[3];
  m.mu_exp = sc[4];
  m.Pr = sc[5];
  m.bulk_ratio = sc[6];
  m.m47 = sc[7];
  m.m48 = sc[8];
  m.ref_species = hd[5];
  m.wide_stencil = hd[6];
  const double dx = sc[9];
  std::vector<double> rhs(nU * n), jvp(nU * n), prod(ns * n), cells(4 * nU);
  int st = oracle_rhs(&m, nx, ny, nz, dx, dx, dx, U.data(), ORC_HYP | ORC_DIFF | ORC_REACT, rhs.data(), 2);
  st |= oracle_rhs_jvp(&m, nx, ny, nz, dx, dx, dx, U.data(), wU.data(), wA.data(),
                       ORC_HYP | ORC_DIFF | ORC_REACT, nullptr, jvp.data(), 2);
  st |= oracle_production(&m, n, U.data(), prod.data());
  const int cl[12] = {0, 0, 0, nx - 1, ny - 1, nz - 1, nx / 2, 0, nz - 1, 1, ny / 2, nz / 2};
  st |= oracle_rhs_cells(&m, nx, ny, nz, dx, dx, dx, U.data(), ORC_HYP | ORC_DIFF | ORC_REACT, 4, cl,
                         cells.data(), 2);
  if (st) return 3;
  FILE *o = fopen(argv[2], "wb");
  if (!o) return 2;
  fwrite(rhs.data(), sizeof(double), rhs.size(), o);
  fwrite(jvp.data(), sizeof(double), jvp.size(), o);
  fwrite(prod.data(), sizeof(double), prod.size(), o);
  fwrite(cells.data(), sizeof(double), cells.size(), o);
  fclose(o);
  return 0;
}
