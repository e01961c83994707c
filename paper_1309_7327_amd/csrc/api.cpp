// C-ABI of the narrowsdc library: context, mechanism upload, work plans,
// right-hand-side evaluation and the (multirate) SDC drivers.
//
// The time integrators follow Section 3 of the paper: collocation on
// Gauss-Lobatto nodes with node-to-node integration matrices S built from
// exact integrals of the Lagrange basis (eqs. gaussapp, compact, expsdc);
// MRSDC mode 1 with the coarse term frozen at the coarse node to the left of
// each fine node (eq. mrupdate) and piecewise-polynomial fine integration
// matrices for fine nodes of type (b)/(c).  f(U_0) is recycled across the
// steps of one call.
//
// The adjoint drivers (end of the file) run the vector-Jacobian product of
// the right-hand side and the reverse sweep of single-rate SDC steps, with
// step-start checkpoints and node states recomputed one step at a time.
#include "../../include/narrowsdc.h"

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "adjoint.h"
#include "launch.h"
#include "nsdc_internal.h"

using namespace nsdc;

namespace {

// ------------------------------------------------------------- quadrature
// Legendre polynomial P_n and its derivative at x (three-term recurrence).
void legendre(int n, long double x, long double &p, long double &dp) {
  long double p0 = 1.0L, p1 = x;
  if (n == 0) { p = 1.0L; dp = 0.0L; return; }
  for (int k = 2; k <= n; ++k) {
    long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = n * (x * p1 - p0) / (x * x - 1.0L);
}

// Gauss-Lobatto nodes on [0, 1]: 0, 1 and the roots of P'_{n-1} (Newton from
// the Chebyshev-Lobatto points).
std::vector<long double> gauss_lobatto(int n) {
  std::vector<long double> x(n);
  const int N = n - 1;
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int j = 0; j < n; ++j) {
    long double t = -std::cos(pi * j / N);
    if (j > 0 && j < N) {
      for (int it = 0; it < 100; ++it) {
        // f = P'_N, f' from the Legendre equation: (1-t^2) P''_N = 2t P'_N - N(N+1) P_N
        long double p, dp;
        legendre(N, t, p, dp);
        long double ddp = (2 * t * dp - N * (N + 1) * p) / (1 - t * t);
        long double dx = dp / ddp;
        t -= dx;
        if (std::fabs((double)dx) < 1e-19) break;
      }
    }
    x[j] = 0.5L * (t + 1.0L);
  }
  x[0] = 0.0L;
  x[N] = 1.0L;
  return x;
}

// Gauss-Legendre rule with n points on [-1, 1] (Newton on P_n).
void gauss_legendre(int n, std::vector<long double> &x, std::vector<long double> &w) {
  x.resize(n);
  w.resize(n);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    long double t = std::cos(pi * (i + 0.75L) / (n + 0.5L));
    long double p, dp;
    for (int it = 0; it < 100; ++it) {
      legendre(n, t, p, dp);
      long double dx = p / dp;
      t -= dx;
      if (std::fabs((double)dx) < 1e-19) break;
    }
    legendre(n, t, p, dp);
    x[i] = t;
    w[i] = 2.0L / ((1 - t * t) * dp * dp);
  }
}

// integral over [a, b] of the Lagrange basis polynomial j of `nodes`
long double lagrange_integral(const std::vector<long double> &nodes, int j, long double a,
                              long double b) {
  std::vector<long double> gx, gw;
  gauss_legendre((int)nodes.size(), gx, gw);
  long double sum = 0.0L;
  for (size_t q = 0; q < gx.size(); ++q) {
    long double t = 0.5L * (a + b) + 0.5L * (b - a) * gx[q];
    long double l = 1.0L;
    for (size_t i = 0; i < nodes.size(); ++i)
      if ((int)i != j) l *= (t - nodes[i]) / (nodes[j] - nodes[i]);
    sum += gw[q] * l;
  }
  return 0.5L * (b - a) * sum;
}

// ------------------------------------------------------------ plans
struct Plan {
  std::vector<box_desc> boxes;
  int nbox = 0;
  long long totS = 0, totI = 0;
  BoxDev *d_boxes = nullptr;
  Item *d_items = nullptr;   // interior, stored, ghost, interior-y, interior-z lists back to back
  int nI = 0, nS = 0, nG = 0;
  TileShape tsI{}, tsS{};
  TileShape tsZ{};             // tile of the z stencil pass
  int nZ = 0;                  // its work items
  // the boundary layers (4 cells deep) of the directions with physical
  // boundaries: work items of the boundary variant of the stencil passes
  int nB[3] = {0, 0, 0};
  // (one plane along the direction per tile row, so every wave's cells
  // share their distance from the boundary and the stencil tables' reads
  // are uniform)
  TileShape tsB[3] = {{1, 16, 16}, {64, 1, 4}, {64, 4, 1}};
  int cap = 0;                 // workgroups per launch (0: one per work item)
  double **d_Utab = nullptr;
  std::vector<double *> Uptrs;
  ~Plan() {
    if (d_boxes) (void)hipFree(d_boxes);
    if (d_items) (void)hipFree(d_items);
    if (d_Utab) (void)hipFree(d_Utab);
  }
};

constexpr int NXCD = 8;   // accelerator complex dies of an MI355X

// Reorder a work list for round-robin dispatch of workgroups over the XCDs
// (workgroup b runs on XCD b mod 8) in a grid-stride loop of G workgroups:
// in every round, the workgroups of one XCD take a contiguous run of the
// natural order.
std::vector<Item> xcd_order(const std::vector<Item> &nat, long long G) {
  const long long n = (long long)nat.size();
  std::vector<Item> out(nat.size());
  if (G < 1) G = 1;
  for (long long base = 0; base < n; base += G) {
    const long long m = std::min(G, n - base);
    const long long per = m / NXCD, rem = m % NXCD;
    for (long long b = 0; b < m; ++b) {
      const long long x = b % NXCD, loc = b / NXCD;
      out[base + b] = nat[base + x * per + std::min(x, rem) + loc];
    }
  }
  return out;
}

TileShape default_tile(int nx, int ny, int nz) {
  (void)ny;
  (void)nz;
  if (nx >= 64) return TileShape{64, 4, 1};
  if (nx >= 32) return TileShape{32, 8, 1};
  return TileShape{16, 4, 4};
}

std::string plan_key(int nbox, const box_desc *b, double *const *U, TileShape tI, TileShape tS) {
  std::string k;
  k.reserve(64 * nbox + 64);
  char buf[160];
  snprintf(buf, sizeof buf, "n%d|%d,%d,%d|%d,%d,%d|", nbox, tI.tx, tI.ty, tI.tz, tS.tx, tS.ty, tS.tz);
  k += buf;
  for (int i = 0; i < nbox; ++i) {
    snprintf(buf, sizeof buf, "%d,%d,%d,%.17g,%.17g,%.17g,np%d,%p;", b[i].nx, b[i].ny, b[i].nz, b[i].dx,
             b[i].dy, b[i].dz, b[i].nonperiodic, U ? (void *)U[i] : nullptr);
    k += buf;
  }
  return k;
}

}  // namespace

// Per-kernel HIP-event timers: events are recorded on the launch stream
// around every launch while a profiler is attached to the context.
namespace nsdc {
struct Profiler {
  struct Rec {
    int id;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t get() {
    if (used < pool.size()) return pool[used++];
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    pool.push_back(e);
    ++used;
    return e;
  }
  ~Profiler() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};
void prof_begin(Profiler *p, int id, hipStream_t s) {
  if (!p) return;
  hipEvent_t e = p->get();
  if (!e) return;
  (void)hipEventRecord(e, s);
  p->recs.push_back(Profiler::Rec{id, e, nullptr});
}
void prof_end(Profiler *p, int id, hipStream_t s) {
  (void)id;
  if (!p || p->recs.empty() || p->recs.back().b) return;
  hipEvent_t e = p->get();
  if (!e) return;
  (void)hipEventRecord(e, s);
  p->recs.back().b = e;
}
}  // namespace nsdc

static const char *KERNEL_NAMES[K_NKERNELS] = {
    "prim_to_cons", "ghost",     "prims",     "vgrad",     "dir_x",     "dir_y",
    "dir_z",        "chem",      "sdc_node",  "mr_fine",   "mr_src",    "dir_adj_x",
    "dir_adj_y",    "dir_adj_z", "chem_adj",  "vgrad_adj", "prims_adj", "fold",
    "adj_linalg",   "sdc_resid", "mr2_imp"};

struct sdc_context {
  int device = 0;
  bool has_mech = false;
  DevMech h_mech{};
  DevMech *d_mech = nullptr;
  const Ops *ops = nullptr;
  int *d_err = nullptr;
  std::string msg;
  // rhs_eval scratch
  double *scratch = nullptr;
  size_t scratch_bytes = 0;
  // multirate coefficient tables, one per scheme (kept until the context is
  // destroyed: captured step graphs hold their addresses); d_fine is the
  // current scheme's
  FineCoef *d_fine = nullptr;
  std::string fine_key;
  std::map<std::string, FineCoef *> fine_tabs;
  std::map<std::string, std::unique_ptr<Plan>> plans;
  TileShape forceI{0, 0, 0}, forceS{0, 0, 0};
  int grid_cap = 0;
  std::unique_ptr<Profiler> prof;
  bool smc_stencil = false;
  // autotuned launch shapes per box set (dimensions only)
  struct Tuned {
    TileShape tI, tS;
    int cap;
  };
  std::map<std::string, Tuned> tuned;
  int n_cu = 0;
  // captured step graphs
  bool use_graph = false;
  // SDC residual early exit (single-rate sdc_step): ratio 0 = off
  bool wide = false;                    // wide-stencil second derivatives
  bool fused_fine = true;               // one-kernel multirate fine sub-steps (4 coarse nodes, 4 sub-steps)
  double resid_ratio = 0.0;
  double *d_resid = nullptr;            // [NSDC_RESID_BLOCKS + 1][2 nU max] partial maxima, result
  ResidCtl *d_rctl = nullptr;           // device state of the residual early exit
  bool last_resid = false;              // the last sdc_step call decided its sweeps on the device
  int last_sweeps = 0;                  // sweeps performed by the last sdc_step call (otherwise)
  std::map<std::string, hipGraphExec_t> graphs;
  // rhs_eval_static: this device's copy of the static scratch array, and a
  // pinned staging buffer (allocated here, at creation) through which the
  // work list reaches it; stage_done marks the last upload's completion
  double *static_scratch = nullptr;
  void *stage = nullptr;
  size_t stage_bytes = 0;
  hipEvent_t stage_done = nullptr;
  bool stage_pending = false;
};

// ------------------------------------------------------------ static scratch
// Device memory of rhs_eval_static (its work list, primitives and velocity
// gradients): a file-scope array instead of hipMalloc.  Every GPU the library
// runs on holds its own copy, at its own address, until the process ends.
// Host code uses that address (from hipGetSymbolAddress, kept per device),
// never the array's name, which on the host is only a stand-in.
static __device__ __align__(256) double scratch[NSDC_STATIC_SCRATCH_BYTES / sizeof(double)];

namespace {

std::mutex g_static_mu;
std::map<int, double *> g_static_ptr;

// This GPU's copy of the static scratch array; `device` must be current.
hipError_t static_scratch_address(int device, double **out) {
  std::lock_guard<std::mutex> lock(g_static_mu);
  auto it = g_static_ptr.find(device);
  if (it != g_static_ptr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    *out = nullptr;
    return e != hipSuccess ? e : hipErrorInvalidSymbol;
  }
  g_static_ptr[device] = static_cast<double *>(ptr);
  *out = static_cast<double *>(ptr);
  return hipSuccess;
}

// pinned staging for the work list of rhs_eval_static: 1 MiB holds 65536
// work items (a 48^3 box with the default tiles needs about 3000); longer
// lists are rejected
constexpr size_t STAGE_BYTES = size_t(1) << 20;

}  // namespace

namespace {

// A roctx range over a host scope: rocprofv3 --marker-trace shows the
// library's calls, steps and sweeps around the kernels they enqueue.
struct Range {
  explicit Range(const char *name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range &) = delete;
  Range &operator=(const Range &) = delete;
};

int fail(sdc_context *c, int code, const std::string &m) {
  if (c) c->msg = m;
  return code;
}

// Captured step graphs hold device addresses (plans, coefficient tables,
// the mechanism's kernel instances) and the kernel variants chosen at
// capture; every change of those drops them.
void drop_graphs(sdc_context *c) {
  if (c->graphs.empty()) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();   // no replay may still be running
  for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.second);
  c->graphs.clear();
}

#define HIPCHECK(ctx, expr)                                                                 \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(ctx, SDC_EHIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

int check_box(sdc_context *c, const box_desc *b) {
  if (!b) return fail(c, SDC_EINVAL, "null box");
  if (b->nx < 1 || b->ny < 1 || b->nz < 1) return fail(c, SDC_EINVAL, "box extents must be >= 1");
  if (b->ng != NSDC_NG) return fail(c, SDC_EINVAL, "ghost layers must be 4");
  if (!(b->dx > 0) || !(b->dy > 0) || !(b->dz > 0)) return fail(c, SDC_EINVAL, "grid spacing must be > 0");
  if (b->nonperiodic & ~7) return fail(c, SDC_EINVAL, "nonperiodic takes bits 1 (x), 2 (y), 4 (z)");
  const int dims[3] = {b->nx, b->ny, b->nz};
  for (int d = 0; d < 3; ++d)
    if (((b->nonperiodic >> d) & 1) && dims[d] < 8)
      return fail(c, SDC_EINVAL, "a direction with physical boundaries needs at least 8 cells");
  if (b->nonperiodic && c->wide)
    return fail(c, SDC_EINVAL, "physical boundaries need the narrow stencil (set_wide_stencil(0))");
  const long long s = (long long)(b->nx + 8) * (b->ny + 8) * (b->nz + 8);
  if (s >= (1LL << 28)) return fail(c, SDC_EINVAL, "box too large (stored cells must be < 2^28)");
  return SDC_OK;
}

// Build (or fetch) the work plan of a set of boxes.
std::string box_signature(int nbox, const box_desc *b) {
  std::string k;
  char buf[64];
  for (int i = 0; i < nbox; ++i) {
    snprintf(buf, sizeof buf, "%d,%d,%d,%d;", b[i].nx, b[i].ny, b[i].nz, b[i].nonperiodic);
    k += buf;
  }
  return k;
}

// Tile shapes and persistent-grid size of a box set: forced by sdc_set_tiles,
// autotuned, or the defaults.
void plan_shape(const sdc_context *c, int nbox, const box_desc *bx, TileShape &tI, TileShape &tS, int &cap) {
  // batches run as persistent launches: a few workgroups per compute unit
  // walk the (box, tile) list
  cap = nbox > 1 ? 4 * std::max(c->n_cu, 1) : 0;
  const bool forced = c->forceI.tx || c->forceS.tx;
  auto tu = forced ? c->tuned.end() : c->tuned.find(box_signature(nbox, bx));
  if (tu != c->tuned.end()) {
    tI = tu->second.tI;
    tS = tu->second.tS;
    cap = tu->second.cap;
    return;
  }
  int mx = 0, my = 0, mz = 0;
  for (int i = 0; i < nbox; ++i) {
    mx = std::max(mx, bx[i].nx);
    my = std::max(my, bx[i].ny);
    mz = std::max(mz, bx[i].nz);
  }
  if (nbox > 1) mx = 16;   // batches: one tile shape for every box
  // a shape forced by sdc_set_tiles replaces the default; a zero shape
  // leaves its index space automatic
  tI = c->forceI.tx ? c->forceI : default_tile(mx, my, mz);
  tS = c->forceS.tx ? c->forceS : default_tile(nbox > 1 ? 16 : mx + 8, my + 8, mz + 8);
}

// Host side of a work plan for p->boxes with p's tile shapes: the per-box
// descriptors and the work lists (interior, stored, ghost, interior with y
// fastest, z-pass tiles), each in XCD order, back to back.
void plan_layout(const sdc_context *c, Plan *p, std::vector<BoxDev> &hb, std::vector<Item> &all) {
  const int nbox = p->nbox;
  const box_desc *bx = p->boxes.data();
  const TileShape tI = p->tsI, tS = p->tsS;
  // the z pass takes the interior tile with its y and z extents exchanged:
  // its waves then share the z-lines' planes
  const TileShape tZ{tI.tx, tI.tz, tI.ty};
  p->tsZ = tZ;
  p->totS = p->totI = 0;
  hb.assign(nbox, BoxDev{});
  std::vector<Item> iI, iS, iG, iY, iZ, iB[3];
  for (int b = 0; b < nbox; ++b) {
    BoxDev &d = hb[b];
    d.nx = bx[b].nx; d.ny = bx[b].ny; d.nz = bx[b].nz;
    d.sx = d.nx + 2 * NSDC_NG; d.sy = d.ny + 2 * NSDC_NG; d.sz = d.nz + 2 * NSDC_NG;
    d.np = bx[b].nonperiodic;
    d.offS = p->totS;
    d.offI = p->totI;
    const double h[3] = {bx[b].dx, bx[b].dy, bx[b].dz};
    for (int k = 0; k < 3; ++k) {
      d.idx[k] = 1.0 / h[k];
      d.idx2[k] = 1.0 / (h[k] * h[k]);
    }
    p->totS += (long long)d.sx * d.sy * d.sz;
    p->totI += (long long)d.nx * d.ny * d.nz;
    for (int z = 0; z < d.nz; z += tI.tz)
      for (int y = 0; y < d.ny; y += tI.ty)
        for (int x = 0; x < d.nx; x += tI.tx) iI.push_back(Item{b, x, y, z});
    // the same tiles with y, respectively z, varying fastest (the direction
    // kernels along y and z share their stencil halos between neighbours)
    for (int z = 0; z < d.nz; z += tI.tz)
      for (int x = 0; x < d.nx; x += tI.tx)
        for (int y = 0; y < d.ny; y += tI.ty) iY.push_back(Item{b, x, y, z});
    for (int y = 0; y < d.ny; y += tZ.ty)
      for (int x = 0; x < d.nx; x += tZ.tx)
        for (int z = 0; z < d.nz; z += tZ.tz) iZ.push_back(Item{b, x, y, z});
    for (int z = 0; z < d.sz; z += tS.tz)
      for (int y = 0; y < d.sy; y += tS.ty)
        for (int x = 0; x < d.sx; x += tS.tx) iS.push_back(Item{b, x, y, z});
    const long long ng = (long long)d.sx * d.sy * d.sz - (long long)d.nx * d.ny * d.nz;
    for (long long g = 0; g < ng; g += 256) iG.push_back(Item{b, (int)g, 0, 0});
    // boundary layers: the 4 planes at both ends of each direction with
    // physical boundaries (at least 8 cells, so the two sets are disjoint)
    const int n3[3] = {d.nx, d.ny, d.nz};
    for (int dd = 0; dd < 3; ++dd) {
      if (!((d.np >> dd) & 1)) continue;
      const TileShape t = p->tsB[dd];
      const int ext[3] = {t.tx, t.ty, t.tz};
      for (int side = 0; side < 2; ++side) {
        int lo[3] = {0, 0, 0}, hi[3] = {d.nx, d.ny, d.nz};
        lo[dd] = side ? n3[dd] - 4 : 0;
        hi[dd] = lo[dd] + 4;
        for (int z = lo[2]; z < hi[2]; z += ext[2])
          for (int y = lo[1]; y < hi[1]; y += ext[1])
            for (int x = lo[0]; x < hi[0]; x += ext[0]) iB[dd].push_back(Item{b, x, y, z});
      }
    }
  }
  p->nI = (int)iI.size();
  p->nS = (int)iS.size();
  p->nG = (int)iG.size();
  p->nZ = (int)iZ.size();
  for (int dd = 0; dd < 3; ++dd) p->nB[dd] = (int)iB[dd].size();
  const long long capE = c->grid_cap > 0 ? c->grid_cap : (p->cap > 0 ? p->cap : (1LL << 30));
  all.clear();
  for (const std::vector<Item> *v : {&iI, &iS, &iG, &iY, &iZ, &iB[0], &iB[1], &iB[2]}) {
    const std::vector<Item> o = xcd_order(*v, std::min<long long>((long long)v->size(), capE));
    all.insert(all.end(), o.begin(), o.end());
  }
}

int get_plan(sdc_context *c, int nbox, const box_desc *bx, double *const *U, Plan **out) {
  TileShape tI{}, tS{};
  int cap = 0;
  plan_shape(c, nbox, bx, tI, tS, cap);
  std::string key = plan_key(nbox, bx, U, tI, tS) + "|cap" + std::to_string(cap) + "|gc" +
                    std::to_string(c->grid_cap);
  auto it = c->plans.find(key);
  if (it != c->plans.end()) {
    *out = it->second.get();
    return SDC_OK;
  }
  if (c->plans.size() > 512) {
    drop_graphs(c);
    c->plans.clear();
  }
  auto p = std::make_unique<Plan>();
  p->nbox = nbox;
  p->boxes.assign(bx, bx + nbox);
  p->tsI = tI;
  p->tsS = tS;
  p->cap = cap;
  std::vector<BoxDev> hb;
  std::vector<Item> all;
  plan_layout(c, p.get(), hb, all);
  HIPCHECK(c, hipMalloc(&p->d_boxes, sizeof(BoxDev) * nbox));
  HIPCHECK(c, hipMemcpy(p->d_boxes, hb.data(), sizeof(BoxDev) * nbox, hipMemcpyHostToDevice));
  HIPCHECK(c, hipMalloc(&p->d_items, sizeof(Item) * all.size()));
  HIPCHECK(c, hipMemcpy(p->d_items, all.data(), sizeof(Item) * all.size(), hipMemcpyHostToDevice));
  if (U) {
    p->Uptrs.assign(U, U + nbox);
    HIPCHECK(c, hipMalloc(&p->d_Utab, sizeof(double *) * nbox));
    HIPCHECK(c, hipMemcpy(p->d_Utab, U, sizeof(double *) * nbox, hipMemcpyHostToDevice));
  }
  *out = p.get();
  c->plans[key] = std::move(p);
  return SDC_OK;
}

// Launch context of a plan whose box descriptors and work lists are at
// d_boxes and d_items on the device.
LaunchCtx make_lc_at(sdc_context *c, const Plan *p, BoxDev *d_boxes, Item *d_items, hipStream_t s) {
  LaunchCtx l;
  l.skip = nullptr;
  l.stream = s;
  l.boxes = d_boxes;
  l.itemsI = d_items;
  l.itemsS = d_items + p->nI;
  l.itemsG = d_items + p->nI + p->nS;
  l.itemsD[0] = l.itemsI;
  l.itemsD[1] = l.itemsG + p->nG;
  l.itemsD[2] = l.itemsD[1] + p->nI;
  l.nD[0] = l.nD[1] = p->nI;
  l.nD[2] = p->nZ;
  const Item *bi = l.itemsD[2] + p->nZ;
  for (int d = 0; d < 3; ++d) {
    l.itemsB[d] = bi;
    l.nB[d] = p->nB[d];
    l.tsB[d] = p->tsB[d];
    bi += p->nB[d];
  }
  l.tsD[0] = l.tsD[1] = p->tsI;
  l.tsD[2] = p->tsZ;
  l.nI = p->nI;
  l.nS = p->nS;
  l.nG = p->nG;
  l.tsI = p->tsI;
  l.tsS = p->tsS;
  l.cap = c->grid_cap > 0 ? c->grid_cap : (p->cap > 0 ? p->cap : 1 << 30);
  l.mech = c->d_mech;
  l.ref_species = c->h_mech.ref;
  l.wide = c->wide;
  l.fused_fine = c->fused_fine;
  l.err = c->d_err;
  l.prof = c->prof.get();
  l.smc_stencil = c->smc_stencil;
  return l;
}

LaunchCtx make_lc(sdc_context *c, Plan *p, hipStream_t s) {
  return make_lc_at(c, p, p->d_boxes, p->d_items, s);
}

// One right-hand-side evaluation into F (interior) from U (ghosted).  warm:
// P holds the previous evaluation of the same boxes (its temperatures start
// the Newton solves).
void eval_rhs_g(const Ops *o, const LaunchCtx &l, FRef U, double *P, double *G, FRef F, unsigned parts,
                bool warm = false) {
  o->ghost(l, U);
  // with the chemistry on, the primitives kernel writes F (zeros and the
  // source) and the direction passes add to it; without, the x pass stores
  // into F (bit 8) and nothing clears it first
  const bool react = parts & RHS_REACT, ad = parts & RHS_AD;
  // the direction passes form the mole fractions from Y and the mean
  // molecular weight, and the species enthalpies from T (narrow stencil,
  // correction velocity); the wide and reference-species forms read the
  // stored ones
  const bool store_x = l.wide || l.ref_species >= 0;
  o->prims(l, U, P, F, react ? 2 : (ad ? 0 : 1), warm ? 1 : 0, store_x ? 1 : 0);
  if (parts & RHS_DIFF) o->vgrad(l, P, G);
  if (ad) {
    for (int d = 0; d < 3; ++d) o->dir(l, d, U, P, G, F, (parts & RHS_AD) | (d == 0 && !react ? 8u : 0u));
  }
}

int check_scheme(sdc_context *c, const sdc_scheme *s) {
  if (!s) return fail(c, SDC_EINVAL, "null scheme");
  if (s->n_coarse < 2 || s->n_coarse > 8) return fail(c, SDC_EINVAL, "n_coarse must be in 2..8");
  if (s->sweeps < 1) return fail(c, SDC_EINVAL, "sweeps must be >= 1");
  if (s->n_fine != 0) {
    if (s->n_fine < 2 || s->n_fine > 9 || s->fine_repeat < 1)
      return fail(c, SDC_EINVAL, "n_fine must be 0 or in 2..9, fine_repeat >= 1");
    if ((s->n_fine - 1) * s->fine_repeat > NSDC_MAXFINE - 1)
      return fail(c, SDC_EINVAL, "too many fine sub-steps per coarse interval");
  }
  if (s->mode < 0 || s->mode > 2) return fail(c, SDC_EINVAL, "mode must be 0, 1 or 2");
  if (s->mode == 2) {
    if (s->n_fine == 0) return fail(c, SDC_EINVAL, "multirate mode 2 needs fine nodes (n_fine >= 2)");
    if ((s->n_fine - 1) * s->fine_repeat + 1 > NSDC_MAXFINE)
      return fail(c, SDC_EINVAL, "too many fine nodes per coarse interval");
  }
  return SDC_OK;
}

// workspace layout (doubles), in order: P, G, U buffers, F arrays
struct WsLayout {
  size_t P, G, Ub, F1, F2, A, total;
  int nUb, nF1, nF2, nA;
};

WsLayout ws_layout(const Plan *p, int ns, const sdc_scheme *s) {
  WsLayout w{};
  const int nU = 5 + ns, nP = prim_fields(ns);
  const int M1 = s->n_coarse - 1;
  if (s->n_fine != 0 && s->mode == 2) {
    // mode 2: F1 = chemistry at the coarse nodes (ns per cell), F2 =
    // advection-diffusion at the fine nodes (nU), two state buffers, and the
    // implicit solve's lane slots in A
    const int M2 = M1 * (s->n_fine - 1) * s->fine_repeat;
    w.nUb = 2;
    w.nF1 = 1 + 2 * M1;
    w.nF2 = 1 + 2 * M2;
    // (interior tiles have at most 256 cells)
    const size_t lanes = (size_t)NSDC_MR2_MAXWG * 256;
    size_t off = 0;
    auto take = [&](size_t n) { size_t o = off; off += (n + 31) & ~size_t(31); return o; };
    w.P = take((size_t)p->totS * nP);
    w.G = take((size_t)p->totS * 9);
    w.Ub = take((size_t)p->totS * nU * w.nUb);
    w.F1 = take((size_t)p->totI * ns * w.nF1);
    w.F2 = take((size_t)p->totI * nU * w.nF2);
    w.A = take(lanes * NSDC_MR2_SLOT(ns));
    w.total = off;
    return w;
  }
  const bool mr = s->n_fine != 0;
  const int M2 = mr ? M1 * (s->n_fine - 1) * s->fine_repeat : 0;
  w.nUb = mr ? 1 : 2;
  w.nF1 = 1 + 2 * M1;
  w.nF2 = mr ? 1 + 2 * M2 : 0;
  w.nA = mr ? (s->n_fine - 1) * s->fine_repeat : 0;   // fine sub-steps of one coarse interval
  size_t off = 0;
  auto take = [&](size_t n) { size_t o = off; off += (n + 31) & ~size_t(31); return o; };
  w.P = take((size_t)p->totS * nP);
  w.G = take((size_t)p->totS * 9);
  w.Ub = take((size_t)p->totS * nU * w.nUb);
  w.F1 = take((size_t)p->totI * nU * w.nF1);
  w.F2 = take((size_t)p->totI * ns * w.nF2);
  w.A = take((size_t)p->totI * nU * w.nA);
  w.total = off;
  return w;
}

// multirate coefficient tables for the scheme, uploaded once per scheme
int fine_tables(sdc_context *c, const sdc_scheme *s) {
  char key[64];
  snprintf(key, sizeof key, "%d,%d,%d", s->n_coarse, s->n_fine, s->fine_repeat);
  if (c->d_fine && c->fine_key == key) return SDC_OK;
  auto known = c->fine_tabs.find(key);
  if (known != c->fine_tabs.end()) {
    c->d_fine = known->second;
    c->fine_key = key;
    return SDC_OK;
  }
  const int M1 = s->n_coarse - 1;
  const int r = (s->n_fine - 1) * s->fine_repeat;
  std::vector<long double> t1 = gauss_lobatto(s->n_coarse), g = gauss_lobatto(s->n_fine);
  std::vector<FineCoef> fc(M1);
  for (int p = 0; p < M1; ++p) {
    FineCoef &f = fc[p];
    std::memset(&f, 0, sizeof f);
    f.n1 = M1 + 1;
    f.nq = r;
    f.nfine = s->n_fine;
    // fine nodes of this coarse interval: `repeat` copies of the fine rule
    std::vector<long double> tf(r + 1);
    const long double a = t1[p], b = t1[p + 1];
    for (int rep = 0; rep < s->fine_repeat; ++rep) {
      const long double lo = a + (b - a) * rep / s->fine_repeat;
      const long double hi = a + (b - a) * (rep + 1) / s->fine_repeat;
      for (int j = 0; j < s->n_fine; ++j) tf[rep * (s->n_fine - 1) + j] = lo + (hi - lo) * g[j];
    }
    tf[r] = b;
    for (int q = 0; q < r; ++q) {
      f.dtq[q] = (double)(tf[q + 1] - tf[q]);
      for (int j = 0; j <= M1; ++j) f.S21[q][j] = (double)lagrange_integral(t1, j, tf[q], tf[q + 1]);
      // piece of the fine interpolant containing [t_q, t_{q+1}]
      const int piece = q / (s->n_fine - 1);
      std::vector<long double> loc(tf.begin() + piece * (s->n_fine - 1),
                                   tf.begin() + piece * (s->n_fine - 1) + s->n_fine);
      f.jlo[q] = piece * (s->n_fine - 1);
      for (int j = 0; j < s->n_fine; ++j) f.S22[q][j] = (double)lagrange_integral(loc, j, tf[q], tf[q + 1]);
      if (r == 4)
        for (int j = 0; j < s->n_fine; ++j) f.S22n[q][f.jlo[q] + j] = f.S22[q][j];
    }
  }
  FineCoef *d = nullptr;
  HIPCHECK(c, hipMalloc(&d, sizeof(FineCoef) * M1));
  c->fine_tabs[key] = d;
  HIPCHECK(c, hipMemcpy(d, fc.data(), sizeof(FineCoef) * M1, hipMemcpyHostToDevice));
  c->d_fine = d;
  c->fine_key = key;
  return SDC_OK;
}

// ------------------------------------------------ multirate SDC, mode 2
// Eq. (mrupdate2): chemistry f1 on the coarse nodes, implicit; advection-
// diffusion f2 on the fine nodes, explicit.  In every coarse interval p the
// implicit kernel first solves for f1 at node p+1 (the interval's explicit
// update as forcing, the f2 corrections of the interval lagged), then the
// fine sub-steps evaluate f2 at their left node and update the state.  f1 of
// the step's end state starts the next step; f2 of it is the last sweep's.
int run_mrsdc2(sdc_context *c, Plan *p, FRef Uuser, double dt, int nsteps, const sdc_scheme *s, double *W,
               const WsLayout &L, const LaunchCtx &l) {
  const Ops *o = c->ops;
  const int ns = o->ns, nU = 5 + ns;
  const int M1 = s->n_coarse - 1, K = s->sweeps;
  const int r = (s->n_fine - 1) * s->fine_repeat, M2 = M1 * r;
  // fine nodes of the step and the multirate integration matrices (units of
  // the step): S21 from the coarse interpolant, S22 from the fine piece
  std::vector<long double> t1 = gauss_lobatto(s->n_coarse), g = gauss_lobatto(s->n_fine);
  std::vector<long double> t2(M2 + 1);
  for (int pi = 0; pi < M1; ++pi)
    for (int rep = 0; rep < s->fine_repeat; ++rep) {
      const long double lo = t1[pi] + (t1[pi + 1] - t1[pi]) * rep / s->fine_repeat;
      const long double hi = t1[pi] + (t1[pi + 1] - t1[pi]) * (rep + 1) / s->fine_repeat;
      for (int j = 0; j < s->n_fine; ++j) t2[pi * r + rep * (s->n_fine - 1) + j] = lo + (hi - lo) * g[j];
    }
  t2[M2] = 1.0L;
  std::vector<std::vector<double>> S21(M2, std::vector<double>(M1 + 1)), S22(M2, std::vector<double>(M2 + 1, 0.0));
  std::vector<int> plo(M2);
  for (int q = 0; q < M2; ++q) {
    for (int j = 0; j <= M1; ++j) S21[q][j] = (double)lagrange_integral(t1, j, t2[q], t2[q + 1]);
    const int lo = (q / (s->n_fine - 1)) * (s->n_fine - 1);
    plo[q] = lo;
    std::vector<long double> loc(t2.begin() + lo, t2.begin() + lo + s->n_fine);
    for (int j = 0; j < s->n_fine; ++j) S22[q][lo + j] = (double)lagrange_integral(loc, j, t2[q], t2[q + 1]);
  }
  double *P = W + L.P, *G = W + L.G;
  const long long fS = p->totS * nU, f1I = p->totI * ns, f2I = p->totI * nU;
  FRef Ub[2] = {FRef{W + L.Ub, nullptr}, FRef{W + L.Ub + fS, nullptr}};
  auto F1p = [&](int slot) { return W + L.F1 + f1I * slot; };
  auto F2p = [&](int slot) { return W + L.F2 + f2I * slot; };
  // slots: 0 the step-start value, 1..M (1..M2) and M+1..2M (M2+1..2M2) the
  // two sweeps' values; roles rotate by renaming
  int s10 = 0, s20 = 0;
  std::vector<int> s1A(M1 + 1), s1B(M1 + 1), s2A(M2 + 1), s2B(M2 + 1);
  for (int m = 1; m <= M1; ++m) {
    s1A[m] = m;
    s1B[m] = M1 + m;
  }
  for (int q = 1; q <= M2; ++q) {
    s2A[q] = q;
    s2B[q] = M2 + q;
  }
  o->chem(l, Uuser, F1p(s10));
  eval_rhs_g(o, l, Uuser, P, G, FRef{F2p(s20), nullptr}, RHS_AD);
  std::vector<int> F1old(M1 + 1), F2old(M2 + 1), F1new(M1 + 1), F2new(M2 + 1);
  for (int step = 0; step < nsteps; ++step) {
    for (int j = 0; j <= M1; ++j) F1old[j] = s10;
    for (int q = 0; q <= M2; ++q) F2old[q] = s20;
    for (int k = 0; k < K; ++k) {
      const Range sweep_range("sweep");
      F1new[0] = s10;
      F2new[0] = s20;
      for (int m = 1; m <= M1; ++m) F1new[m] = (k % 2 == 0) ? s1A[m] : s1B[m];
      for (int q = 1; q <= M2; ++q) F2new[q] = (k % 2 == 0) ? s2A[q] : s2B[q];
      const bool last = step == nsteps - 1 && k == K - 1;
      FRef Ucur = Uuser;
      for (int pi = 0; pi < M1; ++pi) {
        // implicit chemistry of the interval: c1, c2 = dt times the sums of
        // the interval's S21 and S22 rows
        Mr2Imp a{};
        a.n1 = M1 + 1;
        for (int j = 0; j <= M1; ++j) {
          double sum = 0.0;
          for (int q = pi * r; q < (pi + 1) * r; ++q) sum += S21[q][j];
          a.F1[j] = F1p(F1old[j]);
          a.c1[j] = dt * sum;
        }
        a.n2 = r + 1;
        for (int jj = 0; jj <= r; ++jj) {
          double sum = 0.0;
          for (int q = pi * r; q < (pi + 1) * r; ++q) sum += S22[q][pi * r + jj];
          a.F2[jj] = F2p(F2old[pi * r + jj]);
          a.c2[jj] = dt * sum;
        }
        a.F1right = F1p(F1old[pi + 1]);
        a.h = (double)(t1[pi + 1] - t1[pi]) * dt;
        a.X = F1p(F1new[pi + 1]);
        a.J = W + L.A;
        o->mr2_imp(l, Ucur, a);
        for (int q = pi * r; q < (pi + 1) * r; ++q) {
          if (q > 0) eval_rhs_g(o, l, Ucur, P, G, FRef{F2p(F2new[q]), nullptr}, RHS_AD, true);
          const FRef Unext = (k == K - 1 && q == M2 - 1) ? Uuser : Ub[q % 2];
          Mr2Node nd{};
          nd.n2 = s->n_fine;
          for (int j = 0; j < s->n_fine; ++j) {
            nd.F2[j] = F2p(F2old[plo[q] + j]);
            nd.S22[j] = S22[q][plo[q] + j];
          }
          nd.n1 = M1 + 1;
          for (int j = 0; j <= M1; ++j) {
            nd.F1[j] = F1p(F1old[j]);
            nd.S21[j] = S21[q][j];
          }
          nd.F2new_q = F2p(F2new[q]);
          nd.F2old_q = F2p(F2old[q]);
          nd.X = F1p(F1new[pi + 1]);
          nd.F1right = F1p(F1old[pi + 1]);
          nd.dtq = (double)(t2[q + 1] - t2[q]) * dt;
          nd.dt = dt;
          o->mr2_node(l, Ucur, Unext, nd);
          Ucur = Unext;
        }
      }
      if (!last) eval_rhs_g(o, l, Ucur, P, G, FRef{F2p(F2new[M2]), nullptr}, RHS_AD, true);
      F1old = F1new;
      F2old = F2new;
    }
    if (step < nsteps - 1) {
      // f2 of the end state (the last sweep's) by exchanging slot roles; f1
      // of it evaluated afresh into the step-start slot
      const int fin2 = F2new[M2];
      for (int q = 1; q <= M2; ++q) {
        if (s2A[q] == fin2) s2A[q] = s20;
        if (s2B[q] == fin2) s2B[q] = s20;
      }
      s20 = fin2;
      o->ghost(l, Uuser);
      o->chem(l, Uuser, F1p(s10));
    }
  }
  o->ghost(l, Uuser);
  return SDC_OK;
}

int run_sdc(sdc_context *c, Plan *p, FRef Uuser, double dt, int nsteps, const sdc_scheme *s,
            void *ws, size_t ws_bytes, hipStream_t st) {
  const Ops *o = c->ops;
  const int ns = o->ns, nU = 5 + ns;
  const WsLayout L = ws_layout(p, ns, s);
  if (!ws) return fail(c, SDC_EINVAL, "null workspace");
  if (ws_bytes < L.total * sizeof(double)) return fail(c, SDC_ENOMEM, "workspace too small");
  double *W = (double *)ws;
  double *P = W + L.P, *G = W + L.G;
  const LaunchCtx l = make_lc(c, p, st);
  const long long fI = p->totI * nU, fS = p->totS * nU;
  if (s->n_fine != 0 && s->mode == 2) return run_mrsdc2(c, p, Uuser, dt, nsteps, s, W, L, l);
  const int M = s->n_coarse - 1, K = s->sweeps;
  std::vector<long double> t = gauss_lobatto(s->n_coarse);
  if (s->n_fine == 0) {
    // ---------------------------------------------- single-rate SDC
    double Sm[8][8] = {}, dtau[8] = {};
    for (int m = 0; m < M; ++m) {
      dtau[m] = (double)(t[m + 1] - t[m]);
      for (int j = 0; j <= M; ++j) Sm[m][j] = (double)lagrange_integral(t, j, t[m], t[m + 1]);
    }
    double *F0 = W + L.F1;
    double *FA[8], *FB[8];
    for (int m = 1; m <= M; ++m) {
      FA[m] = W + L.F1 + fI * m;
      FB[m] = W + L.F1 + fI * (M + m);
    }
    FRef Ub[2] = {FRef{W + L.Ub, nullptr}, FRef{W + L.Ub + fS, nullptr}};
    // residual early exit (eq. residual): q = last row of the integration
    // matrix, the sum of the node-to-node rows
    // decided on the device: after each sweep but a step's last a kernel
    // measures |R^k| and, once the sweeps stop approaching the collocation
    // solution, sets a flag on which the stage kernels of the step's
    // remaining sweeps return at once; no host synchronisation, so such
    // steps can be captured in a graph too
    const bool resid = c->resid_ratio > 0.0;
    ResidArgs ra{};
    LaunchCtx ls = l;
    ResidCtl *ctl = c->d_rctl;
    if (resid) {
      for (int j = 0; j <= M; ++j)
        for (int m = 0; m < M; ++m) ra.q[j] += Sm[m][j];
      ra.nnodes = M + 1;
      ra.dt = dt;
      ra.partial = c->d_resid;
      ra.out = c->d_resid + (size_t)NSDC_RESID_BLOCKS * 2 * nU;
      ls.skip = &ctl->stop;
      launch_resid_ctl(st, ctl, 0, K);
    }
    eval_rhs_g(o, l, Uuser, P, G, FRef{F0, nullptr}, RHS_ALL);
    for (int step = 0; step < nsteps; ++step) {
      const double *Fold[8];
      for (int j = 0; j <= M; ++j) Fold[j] = F0;
      double *Fnew[8];
      if (resid && step > 0) launch_resid_ctl(st, ctl, 1, K);
      for (int k = 0; k < K; ++k) {
        const Range sweep_range("sweep");
        Fnew[0] = F0;
        for (int m = 1; m <= M; ++m) Fnew[m] = (k % 2 == 0) ? FA[m] : FB[m];
        FRef Ucur = Uuser;
        for (int m = 0; m < M; ++m) {
          if (m > 0) eval_rhs_g(o, ls, Ucur, P, G, FRef{Fnew[m], nullptr}, RHS_ALL, true);
          FRef Unext = (m == M - 1 && k == K - 1) ? Uuser : Ub[m % 2];
          NodeArgs a{};
          for (int j = 0; j <= M; ++j) {
            a.Fold[j] = Fold[j];
            a.S[j] = Sm[m][j];
          }
          a.nnodes = M + 1;
          a.Fnew_m = Fnew[m];
          a.Fold_m = Fold[m];
          a.dtau = dtau[m] * dt;
          a.dt = dt;
          o->sdc_node(ls, Ucur, Unext, a);
          Ucur = Unext;
        }
        const bool last = step == nsteps - 1 && k == K - 1;
        if (!last) eval_rhs_g(o, ls, Ucur, P, G, FRef{Fnew[M], nullptr}, RHS_ALL, true);
        for (int j = 0; j <= M; ++j) Fold[j] = Fnew[j];
        if (resid && k < K - 1) {
          for (int j = 0; j <= M; ++j) ra.F[j] = Fnew[j];
          o->sdc_resid(ls, Uuser, Ucur, ra);
          launch_resid_decide(st, ctl, ra.out, nU, c->resid_ratio, k);
          // if this sweep ended the step, the step returns its end state (in
          // a sweep buffer) and a next step recycles its f(U_M) from the
          // array of the last sweep's, whose roles the host rotates below
          double *Flast = ((K - 1) % 2 == 0) ? FA[M] : FB[M];
          const bool recycle = step < nsteps - 1;
          launch_resid_copy(st, ctl, k, l.boxes, p->nbox, nU, Ucur.base, Uuser, recycle ? Fnew[M] : nullptr,
                            recycle ? Flast : nullptr, recycle ? fI : 0);
        }
      }
      if (resid) launch_resid_ctl(st, ctl, 2, K);
      if (step < nsteps - 1) {
        // recycle f(U_M) as the next step's f(U_0): exchange array roles
        double *fin = Fnew[M];
        double *old0 = F0;
        F0 = fin;
        for (int m = 1; m <= M; ++m) {
          if (FA[m] == fin) FA[m] = old0;
          if (FB[m] == fin) FB[m] = old0;
        }
      }
    }
    o->ghost(l, Uuser);
    return SDC_OK;
  }
  // ------------------------------------------------ multirate SDC, mode 1
  int rc = fine_tables(c, s);
  if (rc) return rc;
  const int r = (s->n_fine - 1) * s->fine_repeat;
  const int M2 = M * r;
  const long long f2I = p->totI * ns;
  // node values live in slots of two arenas: slot 0 holds the step-start
  // value, slots 1..M (1..M2) one sweep's values, M+1..2M (M2+1..2M2) the
  // other's; roles rotate between sweeps and steps by renaming slots.
  double *F1base = W + L.F1, *F2base = W + L.F2;
  auto F1p = [&](int slot) { return F1base + fI * slot; };
  auto F2p = [&](int slot) { return F2base + f2I * slot; };
  int s10 = 0, s20 = 0;
  std::vector<int> s1A(M + 1), s1B(M + 1), s2A(M2 + 1), s2B(M2 + 1);
  for (int m = 1; m <= M; ++m) {
    s1A[m] = m;
    s1B[m] = M + m;
  }
  for (int q = 1; q <= M2; ++q) {
    s2A[q] = q;
    s2B[q] = M2 + q;
  }
  FRef Ucur{W + L.Ub, nullptr};
  eval_rhs_g(o, l, Uuser, P, G, FRef{F1p(s10), nullptr}, RHS_AD);
  o->chem(l, Uuser, F2p(s20));
  std::vector<int> F1old(M + 1), F2old(M2 + 1), F1new(M + 1), F2new(M2 + 1);
  for (int step = 0; step < nsteps; ++step) {
    for (int j = 0; j <= M; ++j) F1old[j] = s10;
    for (int q = 0; q <= M2; ++q) F2old[q] = s20;
    for (int k = 0; k < K; ++k) {
      const Range sweep_range("sweep");
      F1new[0] = s10;
      F2new[0] = s20;
      for (int m = 1; m <= M; ++m) F1new[m] = (k % 2 == 0) ? s1A[m] : s1B[m];
      for (int q = 1; q <= M2; ++q) F2new[q] = (k % 2 == 0) ? s2A[q] : s2B[q];
      const bool last = step == nsteps - 1 && k == K - 1;
      FRef Uout = Ucur;
      for (int pi = 0; pi < M; ++pi) {
        FRef Uin = pi == 0 ? Uuser : Ucur;
        if (pi > 0) eval_rhs_g(o, l, Ucur, P, G, FRef{F1p(F1new[pi]), nullptr}, RHS_AD, true);
        Uout = (k == K - 1 && pi == M - 1) ? Uuser : Ucur;
        FinePtrs fp{};
        fp.F1base = F1base;
        fp.F2base = F2base;
        fp.f1slot = fI;
        fp.f2slot = f2I;
        for (int j = 0; j <= M; ++j) fp.F1old[j] = (unsigned short)F1old[j];
        fp.F1new_p = (unsigned short)F1new[pi];
        fp.F1old_p = (unsigned short)F1old[pi];
        for (int j = 0; j <= r; ++j) {
          fp.F2old[j] = (unsigned short)F2old[pi * r + j];
          fp.F2new[j] = (unsigned short)F2new[pi * r + j];
        }
        fp.q0_known = pi == 0;
        fp.eval_last = (pi == M - 1) && !last;
        fp.nq = r;
        fp.n1 = M + 1;
        fp.dt = dt;
        o->mr_fine(l, Uin, Uout, c->d_fine + pi, fp, W + L.A, fI);
      }
      if (!last) eval_rhs_g(o, l, Uout, P, G, FRef{F1p(F1new[M]), nullptr}, RHS_AD, true);
      F1old = F1new;
      F2old = F2new;
    }
    if (step < nsteps - 1) {
      // recycle f(U_M) as the next step's f(U_0) by exchanging slot roles
      const int fin1 = F1new[M], fin2 = F2new[M2];
      for (int m = 1; m <= M; ++m) {
        if (s1A[m] == fin1) s1A[m] = s10;
        if (s1B[m] == fin1) s1B[m] = s10;
      }
      for (int q = 1; q <= M2; ++q) {
        if (s2A[q] == fin2) s2A[q] = s20;
        if (s2B[q] == fin2) s2B[q] = s20;
      }
      s10 = fin1;
      s20 = fin2;
    }
  }
  o->ghost(l, Uuser);
  return SDC_OK;
}

}  // namespace

// Stencils near a physical boundary (Section 2.5) as weights on the nine
// samples centred on a cell b = 0..3 cells from the boundary: first
// derivatives of the advective terms (sixth- and fourth-order centred for
// b = 3, 2; third order biased away from the boundary for b = 1; one-sided
// third order for b = 0) and of the diffusive terms (the same for b = 3, 2;
// second-order centred for b = 1, one-sided second order for b = 0), and the
// second-derivative pairs as the matrix K of (a u_x)_x h^2 = sum a_o K_oc u_c:
// the sixth-order narrow stencil (Section 2.2, m36 = 281/3600) for b = 3, the
// fourth-order member of the same family for b = 2 (corner entries zero,
// m33 = 1/72), faces (a_i + a_{i+1})(u_{i+1} - u_i)/2 for b = 1, and
// a_0 u'' + a' u' with one-sided second-order differences for b = 0.  The
// boundary above is the mirror image: first-derivative weights reversed and
// negated, K reversed in both indices.
static void boundary_stencils(DevMech &d) {
  std::memset(d.bwA, 0, sizeof d.bwA);
  std::memset(d.bwD, 0, sizeof d.bwD);
  std::memset(d.bK, 0, sizeof d.bK);
  // sample index o = 4 + offset
  auto central = [&](double w[9], const double *c, int n) {
    for (int s = 1; s <= n; ++s) {
      w[4 + s] = c[s - 1];
      w[4 - s] = -c[s - 1];
    }
  };
  const double c6[3] = {3.0 / 4.0, -3.0 / 20.0, 1.0 / 60.0}, c4[2] = {2.0 / 3.0, -1.0 / 12.0};
  central(d.bwA[3], c6, 3);
  central(d.bwD[3], c6, 3);
  central(d.bwA[2], c4, 2);
  central(d.bwD[2], c4, 2);
  d.bwA[1][3] = -2.0 / 6.0; d.bwA[1][4] = -3.0 / 6.0; d.bwA[1][5] = 6.0 / 6.0; d.bwA[1][6] = -1.0 / 6.0;
  d.bwD[1][3] = -0.5; d.bwD[1][5] = 0.5;
  d.bwA[0][4] = -11.0 / 6.0; d.bwA[0][5] = 18.0 / 6.0; d.bwA[0][6] = -9.0 / 6.0; d.bwA[0][7] = 2.0 / 6.0;
  d.bwD[0][4] = -1.5; d.bwD[0][5] = 2.0; d.bwD[0][6] = -0.5;
  // face-sum stencils: H_{i+1/2} = sum_{m,n} a_{i+m} M_{mn} u_{i+n}, K += the
  // face above minus the face below
  auto faces = [&](double K[9][9], const double *M, int lo, int w) {
    for (int m = 0; m < w; ++m)
      for (int n = 0; n < w; ++n) {
        const double v = M[m * w + n];
        K[4 + lo + m][4 + lo + n] += v;
        K[3 + lo + m][3 + lo + n] -= v;
      }
  };
  const double m36 = 281.0 / 3600.0;
  const double q11 = -11.0 / 180 + m36, q12 = 1.0 / 9 - 2 * m36, q13 = -1.0 / 18 + m36, q14 = 1.0 / 180;
  const double q21 = 7.0 / 60 - 3 * m36, q22 = -1.0 / 120 + 5 * m36, q23 = -17.0 / 90 - 2 * m36;
  const double q24 = 5.0 / 72 + m36, q25 = 1.0 / 90 - m36, q31 = -1.0 / 15 + 3 * m36;
  const double q32 = -11.0 / 60 - 3 * m36, q33 = -101.0 / 360, q34 = 137.0 / 180 - 2 * m36;
  const double q35 = -83.0 / 360 + m36;
  const double M6[36] = {q11,  q12,  q13,  q14,  0,    0,    q21,  q22,  q23,  q24,  q25,  0,
                         q31,  q32,  q33,  q34,  q35,  m36,  -m36, -q35, -q34, -q33, -q32, -q31,
                         0,    -q25, -q24, -q23, -q22, -q21, 0,    0,    -q14, -q13, -q12, -q11};
  faces(d.bK[3], M6, -2, 6);
  const double e = 1.0 / 72.0;
  const double M4[16] = {-e,          2 * e + 1.0 / 12, -e - 1.0 / 12,  0,
                         2 * e + 1.0 / 12, -3 * e - 0.75,  2.0 / 3,    e,
                         -e,          -2.0 / 3,      3 * e + 0.75, -2 * e - 1.0 / 12,
                         0,           e + 1.0 / 12,  -2 * e - 1.0 / 12, e};
  faces(d.bK[2], M4, -1, 4);
  const double M2[4] = {-0.5, 0.5, -0.5, 0.5};
  faces(d.bK[1], M2, 0, 2);
  const double c2[9] = {0, 0, 0, 0, 2.0, -5.0, 4.0, -1.0, 0};
  const double c1[9] = {0, 0, 0, 0, -1.5, 2.0, -0.5, 0, 0};
  for (int cc = 0; cc < 9; ++cc) {
    d.bK[0][4][cc] += c2[cc];
    for (int o = 0; o < 9; ++o) d.bK[0][o][cc] += c1[o] * c1[cc];
  }
  for (int b = 0; b < 4; ++b)
    for (int o = 0; o < 9; ++o) {
      d.bwA[4 + b][o] = -d.bwA[b][8 - o];
      d.bwD[4 + b][o] = -d.bwD[b][8 - o];
      for (int cc = 0; cc < 9; ++cc) d.bK[4 + b][o][cc] = d.bK[b][8 - o][8 - cc];
    }
}

// ================================================================ C ABI
extern "C" {

int sdc_context_create(sdc_context **out, int device) {
  if (!out) return SDC_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SDC_EHIP;
  if (hipSetDevice(device) != hipSuccess) return SDC_EHIP;
  auto *c = new sdc_context();
  c->device = device;
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    c->n_cu = 256;
  if (hipMalloc(&c->d_err, sizeof(int)) != hipSuccess || hipMemset(c->d_err, 0, sizeof(int)) != hipSuccess ||
      hipMalloc(&c->d_mech, sizeof(DevMech)) != hipSuccess) {
    delete c;
    return SDC_EHIP;
  }
  // rhs_eval_static's set-up (it allocates nothing itself): this device's
  // static scratch address, the staging buffer and its event.  Failures
  // leave that entry point unavailable (SDC_EHIP) and nothing else.
  if (static_scratch_address(device, &c->static_scratch) != hipSuccess) c->static_scratch = nullptr;
  if (hipHostMalloc(&c->stage, STAGE_BYTES, hipHostMallocDefault) == hipSuccess)
    c->stage_bytes = STAGE_BYTES;
  else
    c->stage = nullptr;
  if (hipEventCreateWithFlags(&c->stage_done, hipEventDisableTiming) != hipSuccess) c->stage_done = nullptr;
  (void)hipGetLastError();
  *out = c;
  return SDC_OK;
}

int sdc_context_destroy(sdc_context *c) {
  if (!c) return SDC_EINVAL;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  drop_graphs(c);
  c->plans.clear();
  if (c->d_err) (void)hipFree(c->d_err);
  if (c->d_mech) (void)hipFree(c->d_mech);
  if (c->scratch) (void)hipFree(c->scratch);
  for (auto &f : c->fine_tabs) (void)hipFree(f.second);
  c->fine_tabs.clear();
  c->d_fine = nullptr;
  if (c->d_resid) (void)hipFree(c->d_resid);
  if (c->d_rctl) (void)hipFree(c->d_rctl);
  if (c->stage_done) (void)hipEventDestroy(c->stage_done);
  if (c->stage) (void)hipHostFree(c->stage);
  delete c;
  return SDC_OK;
}

int sdc_species_supported(int ns) { return ops_for(ns) ? 1 : 0; }

int set_mechanism(sdc_context *c, const mechanism_desc *m) {
  if (!c || !m) return fail(c, SDC_EINVAL, "null argument");
  const Ops *o = ops_for(m->ns);
  if (!o) {
#define NSDC_COUNT_STR(n) " " #n
    return fail(c, SDC_EINVAL, "species count not among those the library was built for:" NSDC_SPECIES_COUNTS(
                                   NSDC_COUNT_STR));
#undef NSDC_COUNT_STR
  }
  if (m->nr < 0 || m->nr > NSDC_NRMAX) return fail(c, SDC_EINVAL, "too many reactions");
  if (!m->W || !m->nasa || !m->Le || (m->nr > 0 && (!m->A || !m->b || !m->Ea || !m->nu_f || !m->nu_r)))
    return fail(c, SDC_EINVAL, "null mechanism array");
  if (!(m->Tlo > 0) || !(m->Thi > m->Tlo)) return fail(c, SDC_EINVAL, "bad temperature range");
  drop_graphs(c);
  DevMech &d = c->h_mech;
  std::memset(&d, 0, sizeof d);
  d.ns = m->ns;
  d.nr = m->nr;
  d.Tlo = m->Tlo;
  d.Thi = m->Thi;
  d.mu_ref = m->mu_ref;
  d.inv_Tref = 1.0 / m->T_ref;
  d.mu_exp = m->mu_exp;
  d.inv_Pr = 1.0 / m->Pr;
  d.bulk = m->bulk_ratio;
  for (int k = 0; k < m->ns; ++k) {
    if (!(m->W[k] > 0) || !(m->Le[k] > 0)) return fail(c, SDC_EINVAL, "bad W or Le");
    d.W[k] = m->W[k];
    d.invW[k] = 1.0 / m->W[k];
    d.Rk[k] = RU / m->W[k];
    d.invLe[k] = 1.0 / m->Le[k];
    const double *a = m->nasa + 7 * k;
    for (int i = 0; i < 5; ++i) {
      d.cp[k][i] = a[i];
      d.hc[k][i] = a[i] / (i + 1);
    }
    d.h6[k] = a[5];
    for (int i = 0; i < 4; ++i) d.sc[k][i] = a[i + 1] / (i + 1);
    d.s7[k] = a[6];
    d.gc[k][0] = a[0] - a[6];
    d.gc[k][1] = -a[1] / 2.0;
    d.gc[k][2] = -a[2] / 6.0;
    d.gc[k][3] = -a[3] / 12.0;
    d.gc[k][4] = -a[4] / 20.0;
  }
  for (int j = 0; j < 64; ++j) d.e2tab[j] = (double)exp2l((long double)j / 64.0L);
  for (int j = 0; j < m->nr; ++j) {
    if (!(m->A[j] > 0)) return fail(c, SDC_EINVAL, "pre-exponential must be > 0");
    d.lnA[j] = std::log(m->A[j]);
    d.beta[j] = m->b[j];
    d.EaR[j] = m->Ea[j] / RU;
    int nr_ = 0, np_ = 0, dnu = 0;
    d.rs[j][0] = d.rs[j][1] = d.ps[j][0] = d.ps[j][1] = -1;
    for (int k = 0; k < m->ns; ++k) {
      const int f = m->nu_f[j * m->ns + k], r = m->nu_r[j * m->ns + k];
      if (f < 0 || r < 0) return fail(c, SDC_EINVAL, "negative stoichiometric coefficient");
      for (int i = 0; i < f; ++i) {
        if (nr_ == 2) return fail(c, SDC_EINVAL, "more than two reactant molecules");
        d.rs[j][nr_++] = k;
      }
      for (int i = 0; i < r; ++i) {
        if (np_ == 2) return fail(c, SDC_EINVAL, "more than two product molecules");
        d.ps[j][np_++] = k;
      }
      dnu += r - f;
    }
    if (nr_ == 0 || np_ == 0) return fail(c, SDC_EINVAL, "reaction without reactants or products");
    // absent second molecules point at the dummy species slot ns
    for (int i = nr_; i < 2; ++i) d.rs[j][i] = m->ns;
    for (int i = np_; i < 2; ++i) d.ps[j][i] = m->ns;
    d.dnu[j] = dnu;
    // the reactants' Gibbs energies folded into the forward rate's exponent
    double *x = d.xc[j];
    x[0] = d.lnA[j];
    x[1] = d.beta[j];
    x[2] = -d.EaR[j];
    x[3] = x[4] = x[5] = x[6] = x[7] = 0.0;
    for (int i = 0; i < 2; ++i) {
      const int k = d.rs[j][i];
      if (k == m->ns) {   // the dummy slot: G = -ln T - ln(R_u / p_ref)
        x[0] += LN_RU_PREF;
        x[1] += 1.0;
        continue;
      }
      x[0] -= d.gc[k][0];
      x[1] += d.cp[k][0];
      x[2] -= d.h6[k];
      for (int p = 1; p < 5; ++p) x[2 + p] -= d.gc[k][p];
    }
  }
  // eighth-order narrow-stencil matrix M(m47, m48), Section 2.2: rows 1..4
  // as printed, rows 5..8 the negated reversals of rows 4..1.
  const double a47 = m->m47, a48 = m->m48;
  const double top[4][8] = {
      {5.0 / 336 + a48, -83.0 / 3600 - a47 / 5 - 14 * a48 / 5, 299.0 / 50400 + 2 * a47 / 5 + 13 * a48 / 5,
       17.0 / 12600 - a47 / 5 - 4 * a48 / 5, 1.0 / 1120, 0, 0, 0},
      {-11.0 / 560 - 2 * a48, -31.0 / 360 + a47 + 3 * a48, 41.0 / 200 - 9 * a47 / 5 + 4 * a48 / 5,
       -5927.0 / 50400 + 4 * a47 / 5 - 9 * a48 / 5, 17.0 / 600 - a47 / 5 - 4 * a48 / 5,
       -503.0 / 50400 + a47 / 5 + 4 * a48 / 5, 0, 0},
      {-1.0 / 280, 1097.0 / 5040 - 2 * a47 + 6 * a48, -1349.0 / 10080 + 3 * a47 - 12 * a48,
       -887.0 / 5040 - a47 + 6 * a48, 3613.0 / 50400 + 4 * a47 / 5 - 9 * a48 / 5,
       467.0 / 25200 - 3 * a47 / 5 + 18 * a48 / 5, 139.0 / 25200 - a47 / 5 - 9 * a48 / 5, 0},
      {17.0 / 1680 + 2 * a48, -319.0 / 2520 + 2 * a47 - 8 * a48, -919.0 / 5040 - 2 * a47 + 6 * a48,
       -445.0 / 2016, 583.0 / 720 - a47 + 6 * a48, -65.0 / 224 - 7 * a48, a47, a48},
  };
  for (int r = 0; r < 4; ++r)
    for (int col = 0; col < 8; ++col) {
      d.M[r][col] = top[r][col];
      d.M[7 - r][7 - col] = -top[r][col];
    }
  for (int o = 0; o < 9; ++o)
    for (int col = 0; col < 9; ++col)
      d.B[o][col] = ((o >= 1 && col >= 1) ? d.M[o - 1][col - 1] : 0.0) - ((o <= 7 && col <= 7) ? d.M[o][col] : 0.0);
  boundary_stencils(d);
  // a new mechanism starts in the correction-velocity form
  d.ref = -1;
  HIPCHECK(c, hipSetDevice(c->device));
  HIPCHECK(c, hipMemcpy(c->d_mech, &d, sizeof d, hipMemcpyHostToDevice));
  c->ops = o;
  c->has_mech = true;
  c->smc_stencil = m->m47 == 3557.0 / 44100.0 && m->m48 == -2083.0 / 117600.0;
  return SDC_OK;
}

int prim_to_cons(sdc_context *c, const box_desc *box, const double *p, const double *T,
                 const double *Y, const double *u, double *U, void *stream) {
  if (!c) return SDC_EINVAL;
  if (!c->has_mech) return fail(c, SDC_ENOMECH, "no mechanism set");
  int rc = check_box(c, box);
  if (rc) return rc;
  if (!p || !T || !Y || !u || !U) return fail(c, SDC_EINVAL, "null field pointer");
  HIPCHECK(c, hipSetDevice(c->device));
  Plan *pl;
  rc = get_plan(c, 1, box, nullptr, &pl);
  if (rc) return rc;
  const LaunchCtx l = make_lc(c, pl, (hipStream_t)stream);
  c->ops->prim_to_cons(l, p, T, Y, u, FRef{U, nullptr});
  c->ops->ghost(l, FRef{U, nullptr});
  HIPCHECK(c, hipGetLastError());
  return SDC_OK;
}

int rhs_eval(sdc_context *c, const box_desc *box, double *U, double *dUdt, unsigned parts,
             void *stream) {
  if (!c) return SDC_EINVAL;
  if (!c->has_mech) return fail(c, SDC_ENOMECH, "no mechanism set");
  int rc = check_box(c, box);
  if (rc) return rc;
  if (!U || !dUdt) return fail(c, SDC_EINVAL, "null field pointer");
  if (parts == 0 || (parts & ~7u)) return fail(c, SDC_EINVAL, "bad parts mask");
  HIPCHECK(c, hipSetDevice(c->device));
  Plan *pl;
  rc = get_plan(c, 1, box, nullptr, &pl);
  if (rc) return rc;
  const int ns = c->ops->ns;
  const size_t need = ((size_t)pl->totS * (prim_fields(ns) + 9) + 64) * sizeof(double);
  if (need > c->scratch_bytes) {
    HIPCHECK(c, hipStreamSynchronize((hipStream_t)stream));
    if (c->scratch) (void)hipFree(c->scratch);
    c->scratch = nullptr;
    c->scratch_bytes = 0;
    HIPCHECK(c, hipMalloc(&c->scratch, need));
    c->scratch_bytes = need;
  }
  double *P = c->scratch;
  double *G = P + ((((size_t)pl->totS * prim_fields(ns)) + 31) & ~size_t(31));
  const Range range("rhs_eval");
  const LaunchCtx l = make_lc(c, pl, (hipStream_t)stream);
  eval_rhs_g(c->ops, l, FRef{U, nullptr}, P, G, FRef{dUdt, nullptr}, parts);
  HIPCHECK(c, hipGetLastError());
  return SDC_OK;
}

int rhs_eval_static(sdc_context *c, const box_desc *box, double *U, double *dUdt, unsigned parts,
                    void *stream) {
  if (!c) return SDC_EINVAL;
  if (!c->has_mech) return fail(c, SDC_ENOMECH, "no mechanism set");
  int rc = check_box(c, box);
  if (rc) return rc;
  if (!U || !dUdt) return fail(c, SDC_EINVAL, "null field pointer");
  if (parts == 0 || (parts & ~7u)) return fail(c, SDC_EINVAL, "bad parts mask");
  HIPCHECK(c, hipSetDevice(c->device));
  if (!c->static_scratch || !c->stage || !c->stage_done)
    return fail(c, SDC_EHIP, "static scratch unavailable on this device");
  // the work plan's host side only; its device lists go to the scratch
  Plan p;
  p.nbox = 1;
  p.boxes.assign(box, box + 1);
  plan_shape(c, 1, box, p.tsI, p.tsS, p.cap);
  std::vector<BoxDev> hb;
  std::vector<Item> items;
  plan_layout(c, &p, hb, items);
  const int ns = c->ops->ns;
  auto up256 = [](size_t n) { return (n + 255) & ~size_t(255); };
  const size_t off_items = up256(sizeof(BoxDev));
  const size_t off_P = up256(off_items + sizeof(Item) * items.size());
  const size_t off_G = up256(off_P + sizeof(double) * (size_t)p.totS * prim_fields(ns));
  const size_t need = off_G + sizeof(double) * ((size_t)p.totS * 9 + 64);
  if (need > NSDC_STATIC_SCRATCH_BYTES)
    return fail(c, SDC_EINVAL, "box needs " + std::to_string(need) + " bytes of static scratch, more than its " +
                                   std::to_string((size_t)NSDC_STATIC_SCRATCH_BYTES) + " (use rhs_eval)");
  if (off_P > c->stage_bytes) return fail(c, SDC_EINVAL, "work list longer than the staging buffer");
  hipStream_t st = (hipStream_t)stream;
  // the previous call's upload must have left the staging buffer
  if (c->stage_pending) HIPCHECK(c, hipEventSynchronize(c->stage_done));
  char *stage = static_cast<char *>(c->stage);
  std::memcpy(stage, hb.data(), sizeof(BoxDev));
  std::memcpy(stage + off_items, items.data(), sizeof(Item) * items.size());
  char *base = reinterpret_cast<char *>(c->static_scratch);
  HIPCHECK(c, hipMemcpyAsync(base, stage, off_P, hipMemcpyHostToDevice, st));
  HIPCHECK(c, hipEventRecord(c->stage_done, st));
  c->stage_pending = true;
  LaunchCtx l = make_lc_at(c, &p, reinterpret_cast<BoxDev *>(base), reinterpret_cast<Item *>(base + off_items), st);
  l.prof = nullptr;   // the profiler's events are created on demand
  eval_rhs_g(c->ops, l, FRef{U, nullptr}, reinterpret_cast<double *>(base + off_P),
             reinterpret_cast<double *>(base + off_G), FRef{dUdt, nullptr}, parts);
  HIPCHECK(c, hipGetLastError());
  return SDC_OK;
}

int sdc_workspace_size(const sdc_context *c, int nbox, const box_desc *boxes,
                       const sdc_scheme *scheme, size_t *bytes) {
  if (!c || !bytes || nbox < 1 || !boxes) return SDC_EINVAL;
  if (!c->has_mech) return SDC_ENOMECH;
  sdc_context *cc = const_cast<sdc_context *>(c);
  for (int i = 0; i < nbox; ++i)
    if (check_box(cc, boxes + i)) return SDC_EINVAL;
  if (check_scheme(cc, scheme)) return SDC_EINVAL;
  Plan p;
  for (int i = 0; i < nbox; ++i) {
    p.totS += (long long)(boxes[i].nx + 8) * (boxes[i].ny + 8) * (boxes[i].nz + 8);
    p.totI += (long long)boxes[i].nx * boxes[i].ny * boxes[i].nz;
  }
  *bytes = ws_layout(&p, c->ops->ns, scheme).total * sizeof(double);
  return SDC_OK;
}

}  // extern "C"

namespace {
// Run (or replay) one sdc_step call.  With graphs enabled and a non-null
// stream the launches of the whole call are captured once into a HIP graph,
// keyed by everything they depend on, and replayed on identical calls.
int step_entry(sdc_context *c, int nbox, const box_desc *boxes, double *const *U, double dt,
               int nsteps, const sdc_scheme *scheme, void *workspace, size_t ws_bytes,
               hipStream_t stream) {
  const Range range(nbox > 1 ? "sdc_step_batched" : "sdc_step");
  if (c->resid_ratio > 0.0 && scheme->n_fine != 0)
    return fail(c, SDC_EINVAL, "the residual early exit covers single-rate schemes only");
  c->last_resid = c->resid_ratio > 0.0;
  c->last_sweeps = scheme->sweeps * nsteps;
  Plan *pl;
  int rc = get_plan(c, nbox, boxes, nbox > 1 ? U : nullptr, &pl);
  if (rc) return rc;
  FRef Uref = nbox > 1 ? FRef{nullptr, pl->d_Utab} : FRef{U[0], nullptr};
  if (scheme->n_fine != 0 && scheme->mode != 2) {
    rc = fine_tables(c, scheme);
    if (rc) return rc;
  }
  if (!c->use_graph || !stream || c->prof) {
    rc = run_sdc(c, pl, Uref, dt, nsteps, scheme, workspace, ws_bytes, stream);
    if (rc) return rc;
    HIPCHECK(c, hipGetLastError());
    return SDC_OK;
  }
  // the key names everything the captured launches depend on: the plan, the
  // scheme and its coefficient table, the state and workspace addresses and
  // the kernel variants (species count, stencil, species-diffusion form,
  // fine-sweep form)
  char buf[320];
  const bool tables = scheme->n_fine != 0 && scheme->mode != 2;
  snprintf(buf, sizeof buf, "|%p|%.17g|%d|%d,%d,%d,%d,m%d|%p|%zu|%p|ns%d|w%d|ref%d|ff%d|smc%d|%p|rr%.17g", (void *)pl,
           dt, nsteps, scheme->n_coarse, scheme->sweeps, scheme->n_fine, scheme->fine_repeat,
           scheme->mode == 2 ? 2 : 1, workspace, ws_bytes, nbox > 1 ? nullptr : (void *)U[0], c->ops->ns,
           (int)c->wide, c->h_mech.ref, (int)c->fused_fine, (int)c->smc_stencil,
           tables ? (void *)c->d_fine : nullptr, c->resid_ratio);
  const std::string key = buf;
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    if (c->graphs.size() >= 8) drop_graphs(c);
    HIPCHECK(c, hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    rc = run_sdc(c, pl, Uref, dt, nsteps, scheme, workspace, ws_bytes, stream);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(stream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail(c, SDC_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(c, SDC_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    it = c->graphs.emplace(key, exec).first;
  }
  HIPCHECK(c, hipGraphLaunch(it->second, stream));
  return SDC_OK;
}
}  // namespace

extern "C" {

int sdc_step(sdc_context *c, const box_desc *box, double *U, double dt, int nsteps,
             const sdc_scheme *scheme, void *workspace, size_t ws_bytes, void *stream) {
  if (!c) return SDC_EINVAL;
  if (!c->has_mech) return fail(c, SDC_ENOMECH, "no mechanism set");
  int rc = check_box(c, box);
  if (rc) return rc;
  rc = check_scheme(c, scheme);
  if (rc) return rc;
  if (!U) return fail(c, SDC_EINVAL, "null state");
  if (!(dt > 0) || nsteps < 1) return fail(c, SDC_EINVAL, "dt must be > 0 and nsteps >= 1");
  HIPCHECK(c, hipSetDevice(c->device));
  double *Ut[1] = {U};
  return step_entry(c, 1, box, Ut, dt, nsteps, scheme, workspace, ws_bytes, (hipStream_t)stream);
}

int sdc_step_batched(sdc_context *c, int nbox, const box_desc *boxes, double *const *U, double dt,
                     int nsteps, const sdc_scheme *scheme, void *workspace, size_t ws_bytes,
                     void *stream) {
  if (!c) return SDC_EINVAL;
  if (!c->has_mech) return fail(c, SDC_ENOMECH, "no mechanism set");
  if (nbox < 1 || !boxes || !U) return fail(c, SDC_EINVAL, "bad batch");
  for (int i = 0; i < nbox; ++i) {
    int rc = check_box(c, boxes + i);
    if (rc) return rc;
    if (!U[i]) return fail(c, SDC_EINVAL, "null state");
  }
  int rc = check_scheme(c, scheme);
  if (rc) return rc;
  if (!(dt > 0) || nsteps < 1) return fail(c, SDC_EINVAL, "dt must be > 0 and nsteps >= 1");
  HIPCHECK(c, hipSetDevice(c->device));
  return step_entry(c, nbox, boxes, U, dt, nsteps, scheme, workspace, ws_bytes, (hipStream_t)stream);
}

int set_wide_stencil(sdc_context *c, int enable) {
  if (!c) return SDC_EINVAL;
  if (c->wide != (enable != 0)) drop_graphs(c);
  c->wide = enable != 0;
  return SDC_OK;
}

int sdc_set_fused_fine(sdc_context *c, int enable) {
  if (!c) return SDC_EINVAL;
  if (c->fused_fine != (enable != 0)) drop_graphs(c);
  c->fused_fine = enable != 0;
  return SDC_OK;
}

int sdc_set_residual_exit(sdc_context *c, double ratio) {
  if (!c) return SDC_EINVAL;
  if (!(ratio == 0.0 || ratio > 1.0)) return fail(c, SDC_EINVAL, "residual ratio must be 0 (off) or > 1");
  if (ratio > 0.0 && !c->d_resid) {
    HIPCHECK(c, hipSetDevice(c->device));
    HIPCHECK(c, hipMalloc(&c->d_resid, sizeof(double) * (NSDC_RESID_BLOCKS + 1) * 2 * (5 + NSDC_NSMAX)));
    HIPCHECK(c, hipMalloc(&c->d_rctl, sizeof(ResidCtl)));
    HIPCHECK(c, hipMemset(c->d_rctl, 0, sizeof(ResidCtl)));
  }
  c->resid_ratio = ratio;
  return SDC_OK;
}

int sdc_residual_history(const sdc_context *c, int max, double *norms, int *count, int *sweeps) {
  if (!c || max < 0 || (max > 0 && !norms)) return SDC_EINVAL;
  if (!c->last_resid) {
    if (count) *count = 0;
    if (sweeps) *sweeps = c->last_sweeps;
    return SDC_OK;
  }
  // the decisions live on the device: wait for the call, then read them
  if (hipSetDevice(c->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return SDC_EHIP;
  ResidCtl h;
  if (hipMemcpy(&h, c->d_rctl, sizeof h, hipMemcpyDeviceToHost) != hipSuccess) return SDC_EHIP;
  const int n = std::min(h.count, NSDC_RESID_HIST);
  for (int i = 0; i < n && i < max; ++i) norms[i] = h.hist[i];
  if (count) *count = n;
  if (sweeps) *sweeps = h.sweeps;
  return SDC_OK;
}

int sdc_set_graph(sdc_context *c, int enable) {
  if (!c) return SDC_EINVAL;
  c->use_graph = enable != 0;
  if (!enable) drop_graphs(c);
  return SDC_OK;
}

int sdc_autotune(sdc_context *c, int nbox, const box_desc *boxes, double *const *U, void *workspace,
                 size_t ws_bytes, void *stream, int *choice) {
  if (!c) return SDC_EINVAL;
  if (!c->has_mech) return fail(c, SDC_ENOMECH, "no mechanism set");
  if (nbox < 1 || !boxes || !U || !workspace) return fail(c, SDC_EINVAL, "bad batch");
  for (int i = 0; i < nbox; ++i) {
    int rc = check_box(c, boxes + i);
    if (rc) return rc;
  }
  HIPCHECK(c, hipSetDevice(c->device));
  Plan probe;
  for (int i = 0; i < nbox; ++i) {
    probe.totS += (long long)(boxes[i].nx + 8) * (boxes[i].ny + 8) * (boxes[i].nz + 8);
    probe.totI += (long long)boxes[i].nx * boxes[i].ny * boxes[i].nz;
  }
  const sdc_scheme sr{2, 1, 0, 1};
  const WsLayout L = ws_layout(&probe, c->ops->ns, &sr);
  if (ws_bytes < L.total * sizeof(double)) return fail(c, SDC_ENOMEM, "workspace too small for tuning");
  double *W = (double *)workspace;
  double *P = W + L.P, *G = W + L.G, *F = W + L.F1;
  static const TileShape cands[] = {{64, 4, 1}, {32, 8, 1}, {16, 16, 1}, {16, 8, 2}, {16, 4, 4},
                                    {8, 8, 4}, {32, 4, 2}, {64, 2, 2}};
  const int ncand = (int)(sizeof(cands) / sizeof(cands[0]));
  const int caps[] = {0, 2 * std::max(c->n_cu, 1), 4 * std::max(c->n_cu, 1), 8 * std::max(c->n_cu, 1)};
  hipEvent_t e0, e1;
  HIPCHECK(c, hipEventCreate(&e0));
  HIPCHECK(c, hipEventCreate(&e1));
  const TileShape fI = c->forceI, fS = c->forceS;
  const int fcap = c->grid_cap;
  float best = 1e30f;
  int bi = 0, bc = 0;
  hipStream_t st = (hipStream_t)stream;
  std::unique_ptr<Profiler> saved = std::move(c->prof);
  for (int ci = 0; ci < ncand; ++ci)
    for (int k = 0; k < 4; ++k) {
      c->forceI = cands[ci];
      c->forceS = cands[ci];
      c->grid_cap = caps[k];
      Plan *pl;
      int rc = get_plan(c, nbox, boxes, nbox > 1 ? U : nullptr, &pl);
      if (rc) break;
      const LaunchCtx l = make_lc(c, pl, st);
      FRef Uref = nbox > 1 ? FRef{nullptr, pl->d_Utab} : FRef{U[0], nullptr};
      float t = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        (void)hipEventRecord(e0, st);
        eval_rhs_g(c->ops, l, Uref, P, G, FRef{F, nullptr}, RHS_ALL);
        (void)hipEventRecord(e1, st);
        HIPCHECK(c, hipEventSynchronize(e1));
        float ms = 0.0f;
        HIPCHECK(c, hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0) t = std::min(t, ms);
      }
      if (t < best) {
        best = t;
        bi = ci;
        bc = k;
      }
    }
  c->prof = std::move(saved);
  c->forceI = fI;
  c->forceS = fS;
  c->grid_cap = fcap;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->tuned[box_signature(nbox, boxes)] = sdc_context::Tuned{cands[bi], cands[bi], caps[bc]};
  if (choice) {
    choice[0] = cands[bi].tx;
    choice[1] = cands[bi].ty;
    choice[2] = cands[bi].tz;
    choice[3] = caps[bc];
  }
  HIPCHECK(c, hipGetLastError());
  return SDC_OK;
}

int last_status(sdc_context *c, void *stream) {
  if (!c) return SDC_EINVAL;
  HIPCHECK(c, hipSetDevice(c->device));
  HIPCHECK(c, hipStreamSynchronize((hipStream_t)stream));
  int e = 0;
  HIPCHECK(c, hipMemcpy(&e, c->d_err, sizeof e, hipMemcpyDeviceToHost));
  if (e) {
    HIPCHECK(c, hipMemset(c->d_err, 0, sizeof(int)));
    return fail(c, SDC_ETEMP, "device error flags " + std::to_string(e) +
                                  " (1 Newton not converged, 2 T out of range, 4 rho <= 0, 8 implicit chemistry not converged)");
  }
  return SDC_OK;
}

const char *last_error_message(const sdc_context *c) { return c ? c->msg.c_str() : "null context"; }

// Tuning hooks (not part of the documented interface): force the tile
// shapes of the interior and stored index spaces (0 = automatic) and cap the
// grid size of every launch (0 = one workgroup per item).
int sdc_set_tiles(sdc_context *c, int ix, int iy, int iz, int sx, int sy, int sz, int grid_cap) {
  if (!c) return SDC_EINVAL;
  // each shape is all zero (automatic) or all positive
  auto valid = [](int x, int y, int z) { return (x == 0 && y == 0 && z == 0) || (x > 0 && y > 0 && z > 0); };
  if (!valid(ix, iy, iz) || !valid(sx, sy, sz) || grid_cap < 0)
    return fail(c, SDC_EINVAL, "tile extents must be all zero or all positive, grid_cap >= 0");
  if (ix * iy * iz > 256 || sx * sy * sz > 256) return fail(c, SDC_EINVAL, "tile larger than 256 threads");
  if ((ix * iy * iz) % 64 != 0) return fail(c, SDC_EINVAL, "interior tile must be a multiple of 64 threads");
  c->forceI = TileShape{ix, iy, iz};
  c->forceS = TileShape{sx, sy, sz};
  c->grid_cap = grid_cap;
  return SDC_OK;
}

int sdc_profile_enable(sdc_context *c, int enable) {
  if (!c) return SDC_EINVAL;
  if (enable) {
    if (!c->prof) c->prof = std::make_unique<Profiler>();
    c->prof->recs.clear();
    c->prof->used = 0;
  } else {
    c->prof.reset();
  }
  return SDC_OK;
}

int sdc_profile_read(sdc_context *c, void *stream, double *total_ms, int *count) {
  if (!c || !total_ms || !count) return SDC_EINVAL;
  for (int k = 0; k < K_NKERNELS; ++k) {
    total_ms[k] = 0.0;
    count[k] = 0;
  }
  if (!c->prof) return K_NKERNELS;
  HIPCHECK(c, hipStreamSynchronize((hipStream_t)stream));
  for (const auto &r : c->prof->recs) {
    if (!r.b) continue;
    float ms = 0.0f;
    HIPCHECK(c, hipEventElapsedTime(&ms, r.a, r.b));
    total_ms[r.id] += ms;
    count[r.id] += 1;
  }
  c->prof->recs.clear();
  c->prof->used = 0;
  return K_NKERNELS;
}

const char *sdc_kernel_name(int id) { return (id >= 0 && id < K_NKERNELS) ? KERNEL_NAMES[id] : ""; }

}  // extern "C"

// ================================================================ adjoint
namespace {

int grid_cap_of(const sdc_context *c, const Plan *p) {
  return c->grid_cap > 0 ? c->grid_cap : (p->cap > 0 ? p->cap : 1 << 30);
}

// scratch of one vector-Jacobian product (doubles): primitive fields and
// velocity gradient of the forward evaluation, the adjoint accumulators
// (contiguous, cleared together), the per-cell coefficient table of the
// direction adjoints and the ln A partials
struct VjpLayout {
  size_t P, G, Pb, Gb, Ub, coef, part, total;
};
VjpLayout vjp_layout(const Plan *p, int ns, int nr, int cap) {
  VjpLayout w{};
  const int nU = 5 + ns, nP = prim_fields(ns);
  size_t off = 0;
  auto take = [&](size_t n) {
    size_t o = off;
    off += (n + 31) & ~size_t(31);
    return o;
  };
  w.P = take((size_t)p->totS * nP);
  w.G = take((size_t)p->totS * 9);
  w.Pb = take((size_t)p->totS * nP);
  w.Gb = take((size_t)p->totS * 9);
  w.Ub = take((size_t)p->totS * nU);
  w.coef = take((size_t)p->totI * 7);
  const int nblk = std::max(1, std::min(p->nI, cap));
  w.part = take((size_t)nblk * std::max(nr, 1));
  w.total = off;
  return w;
}


// Ubar (interior) += (d rhs/dU)^T V, lnA_bar += (d rhs/d ln A)^T V.
int rhs_vjp_g(sdc_context *c, Plan *p, const LaunchCtx &l, double *U, const double *V, double *Ubar,
              double *lnA_bar, unsigned parts, double *W) {
  const Ops *o = c->ops;
  const AdjOps *a = adj_ops_for(o->ns);
  const int ns = o->ns, nU = 5 + ns;
  const VjpLayout L = vjp_layout(p, ns, c->h_mech.nr, grid_cap_of(c, p));
  double *P = W + L.P, *G = W + L.G;
  const FRef Uf{U, nullptr};
  o->ghost(l, Uf);
  o->prims(l, Uf, P, FRef{nullptr, nullptr}, 0, 0, 1);   // the transposes read X and h
  if (parts & RHS_DIFF) o->vgrad(l, P, G);
  adj_fill0(l, W + L.Pb, (long long)(L.Ub - L.Pb) + (long long)p->totS * nU);
  const AdjBufs ab{W + L.Ub, W + L.Pb, W + L.Gb};
  if (parts & RHS_AD)
    for (int d = 0; d < 3; ++d) a->dir(l, d, U, P, G, V, ab, W + L.coef, parts & RHS_AD);
  int nblk = 0;
  if (parts & RHS_REACT) nblk = a->chem(l, U, V, ab, W + L.part);
  if (parts & RHS_DIFF) a->vgrad(l, ab);
  a->prims(l, U, ab);
  a->fold(l, ab, Ubar);
  if ((parts & RHS_REACT) && lnA_bar && c->h_mech.nr > 0) adj_lnA_reduce(l, W + L.part, nblk, c->h_mech.nr, lnA_bar);
  return SDC_OK;
}

// workspace of the SDC adjoint (doubles): one VJP scratch, the step-start
// checkpoints, the node states of one step, the right-hand sides of the
// recomputation and the adjoint arrays
struct SdcVjpLayout {
  VjpLayout v;
  size_t ckpt, nodes, F, A, total;
};
SdcVjpLayout sdc_vjp_layout(const Plan *p, int ns, int nr, int cap, const sdc_scheme *s, int nsteps) {
  SdcVjpLayout w{};
  w.v = vjp_layout(p, ns, nr, cap);
  const int nU = 5 + ns, M = s->n_coarse - 1, K = s->sweeps;
  const size_t fS = (size_t)p->totS * nU, fI = (size_t)p->totI * nU;
  size_t off = w.v.total;
  w.ckpt = off;
  off += fS * nsteps;
  w.nodes = off;
  off += fS * (size_t)K * M;
  w.F = off;
  off += fI * (2 * M + 1);
  w.A = off;
  off += fI * (4 + 2 * (M + 1));
  w.total = off;
  return w;
}

int check_vjp_args(sdc_context *c, const box_desc *box) {
  if (!c) return SDC_EINVAL;
  if (!c->has_mech) return fail(c, SDC_ENOMECH, "no mechanism set");
  if (c->h_mech.ref >= 0)
    return fail(c, SDC_EINVAL, "the adjoint covers the correction-velocity form of the species diffusion only");
  if (c->resid_ratio > 0.0) return fail(c, SDC_EINVAL, "the adjoint covers fixed sweep counts only");
  if (c->wide) return fail(c, SDC_EINVAL, "the adjoint covers the narrow stencil only");
  int rc = check_box(c, box);
  if (rc) return rc;
  if (box->nonperiodic) return fail(c, SDC_EINVAL, "the adjoint covers periodic boxes only");
  const TileShape t = c->forceI;
  if (t.tx && (t.tx * t.ty * t.tz) % 64) return fail(c, SDC_EINVAL, "interior tile must be a multiple of 64 threads");
  return SDC_OK;
}

void sdc_tables(const sdc_scheme *s, double Sm[8][8], double dtau[8]) {
  std::vector<long double> t = gauss_lobatto(s->n_coarse);
  const int M = s->n_coarse - 1;
  for (int m = 0; m < M; ++m) {
    dtau[m] = (double)(t[m + 1] - t[m]);
    for (int j = 0; j <= M; ++j) Sm[m][j] = (double)lagrange_integral(t, j, t[m], t[m + 1]);
  }
}

// One single-rate SDC step from X (ghosted) with every node state kept:
// node[k M + m - 1] = U^{k+1}_m, m = 1..M (the same launches and arguments
// as the forward driver, so the states are identical).
void sdc_forward_record(const Ops *o, const LaunchCtx &l, double *X, double dt, const sdc_scheme *s,
                        double *P, double *G, double *Fbase, long long fI, long long fS, double *nodes) {
  const int M = s->n_coarse - 1, K = s->sweeps;
  double Sm[8][8] = {}, dtau[8] = {};
  sdc_tables(s, Sm, dtau);
  double *F0 = Fbase;
  double *FA[8], *FB[8];
  for (int m = 1; m <= M; ++m) {
    FA[m] = Fbase + fI * m;
    FB[m] = Fbase + fI * (M + m);
  }
  eval_rhs_g(o, l, FRef{X, nullptr}, P, G, FRef{F0, nullptr}, RHS_ALL);
  const double *Fold[8];
  for (int j = 0; j <= M; ++j) Fold[j] = F0;
  double *Fnew[8];
  for (int k = 0; k < K; ++k) {
    Fnew[0] = F0;
    for (int m = 1; m <= M; ++m) Fnew[m] = (k % 2 == 0) ? FA[m] : FB[m];
    FRef Ucur{X, nullptr};
    for (int m = 0; m < M; ++m) {
      if (m > 0) eval_rhs_g(o, l, Ucur, P, G, FRef{Fnew[m], nullptr}, RHS_ALL, true);
      FRef Unext{nodes + fS * ((long long)k * M + m), nullptr};
      NodeArgs a{};
      for (int j = 0; j <= M; ++j) {
        a.Fold[j] = Fold[j];
        a.S[j] = Sm[m][j];
      }
      a.nnodes = M + 1;
      a.Fnew_m = Fnew[m];
      a.Fold_m = Fold[m];
      a.dtau = dtau[m] * dt;
      a.dt = dt;
      o->sdc_node(l, Ucur, Unext, a);
      Ucur = Unext;
    }
    if (k < K - 1) eval_rhs_g(o, l, Ucur, P, G, FRef{Fnew[M], nullptr}, RHS_ALL, true);
    for (int j = 0; j <= M; ++j) Fold[j] = Fnew[j];
  }
}

// Reverse sweep of nsteps single-rate SDC steps.  For the update
//   U^k_{m+1} = U^k_m + dtau_m (F^k_m - F^{k-1}_m) + dt sum_j S_mj F^{k-1}_j
// (F^k_m = f(U^k_m) for m >= 1, F^k_0 = f(U_0), sweep 0 spreads U_0 and
// f(U_0) to every node) the adjoint R of U^k_{m+1} gives
//   Fb^k_m += dtau_m R,  Fb^{k-1}_j += (dt S_mj - [j = m] dtau_m) R,
//   R(U^k_m) = R + J(U^k_m)^T Fb^k_m   (m >= 1),
// swept from the last sweep and node back to U_0.
int run_sdc_vjp(sdc_context *c, Plan *p, double *U0, double dt, int nsteps, const sdc_scheme *s,
                const double *UNbar, double *U0bar, double *lnA_bar, void *ws, size_t ws_bytes, hipStream_t st) {
  const Ops *o = c->ops;
  const int ns = o->ns, nU = 5 + ns, M = s->n_coarse - 1, K = s->sweeps;
  const SdcVjpLayout L = sdc_vjp_layout(p, ns, c->h_mech.nr, grid_cap_of(c, p), s, nsteps);
  if (!ws) return fail(c, SDC_EINVAL, "null workspace");
  if (ws_bytes < L.total * sizeof(double)) return fail(c, SDC_ENOMEM, "workspace too small");
  double *W = (double *)ws;
  double *P = W + L.v.P, *G = W + L.v.G;
  const LaunchCtx l = make_lc(c, p, st);
  const long long fI = p->totI * nU, fS = p->totS * nU;
  double Sm[8][8] = {}, dtau[8] = {};
  sdc_tables(s, Sm, dtau);
  double *ckpt = W + L.ckpt, *nodes = W + L.nodes, *Fw = W + L.F;
  double *R = W + L.A, *Rout = R + fI, *U0b = R + 2 * fI, *F0b = R + 3 * fI;
  double *Fb = R + 4 * fI, *Fbm = Fb + fI * (M + 1);
  auto node = [&](int k, int m) { return nodes + fS * ((long long)(k - 1) * M + (m - 1)); };
  auto vjp = [&](double *U, const double *V, double *out) {
    return rhs_vjp_g(c, p, l, U, V, out, lnA_bar, RHS_ALL, W);
  };
  // step-start checkpoints
  HIPCHECK(c, hipMemcpyAsync(ckpt, U0, sizeof(double) * fS, hipMemcpyDeviceToDevice, st));
  for (int n = 0; n + 1 < nsteps; ++n) {
    sdc_forward_record(o, l, ckpt + fS * n, dt, s, P, G, Fw, fI, fS, nodes);
    HIPCHECK(c, hipMemcpyAsync(ckpt + fS * (n + 1), node(K, M), sizeof(double) * fS, hipMemcpyDeviceToDevice, st));
  }
  HIPCHECK(c, hipMemcpyAsync(Rout, UNbar, sizeof(double) * fI, hipMemcpyDeviceToDevice, st));
  for (int n = nsteps - 1; n >= 0; --n) {
    sdc_forward_record(o, l, ckpt + fS * n, dt, s, P, G, Fw, fI, fS, nodes);
    adj_fill0(l, U0b, 2 * fI + fI * (M + 1));   // U0b, F0b, Fb
    double *cur = Fb, *prev = Fbm;
    for (int k = K; k >= 1; --k) {
      adj_fill0(l, prev, fI * (M + 1));
      if (k == K) {
        HIPCHECK(c, hipMemcpyAsync(R, Rout, sizeof(double) * fI, hipMemcpyDeviceToDevice, st));
      } else {
        adj_fill0(l, R, fI);
        int rc = vjp(node(k, M), cur + fI * M, R);
        if (rc) return rc;
      }
      for (int m = M - 1; m >= 0; --m) {
        AxpyArgs a{};
        a.nt = M + 2;
        a.Y[0] = cur + fI * m;
        a.c[0] = dtau[m] * dt;
        for (int j = 0; j <= M; ++j) {
          a.Y[1 + j] = prev + fI * j;
          a.c[1 + j] = dt * Sm[m][j] - (j == m ? dtau[m] * dt : 0.0);
        }
        adj_axpy(l, R, a, fI);
        if (m >= 1) {
          int rc = vjp(node(k, m), cur + fI * m, R);
          if (rc) return rc;
        } else {
          AxpyArgs u{};
          u.nt = 1;
          u.Y[0] = U0b;
          u.c[0] = 1.0;
          adj_axpy(l, R, u, fI);
          u.Y[0] = F0b;
          adj_axpy(l, cur, u, fI);
        }
      }
      std::swap(cur, prev);
    }
    // sweep 0: every node value of the first sweep's "old" iterate is f(U_0)
    LincombArgs lc{};
    lc.nt = M + 2;
    lc.X[0] = F0b;
    lc.c[0] = 1.0;
    for (int j = 0; j <= M; ++j) {
      lc.X[1 + j] = cur + fI * j;
      lc.c[1 + j] = 1.0;
    }
    adj_lincomb(l, lc, F0b, fI);
    HIPCHECK(c, hipMemcpyAsync(Rout, U0b, sizeof(double) * fI, hipMemcpyDeviceToDevice, st));
    int rc = vjp(ckpt + fS * n, F0b, Rout);
    if (rc) return rc;
  }
  HIPCHECK(c, hipMemcpyAsync(U0bar, Rout, sizeof(double) * fI, hipMemcpyDeviceToDevice, st));
  return SDC_OK;
}

}  // namespace

extern "C" {

int rhs_vjp(sdc_context *c, const box_desc *box, double *U, const double *dUdt_bar, double *U_bar,
            double *lnA_bar, unsigned parts, void *stream) {
  int rc = check_vjp_args(c, box);
  if (rc) return rc;
  if (!U || !dUdt_bar || !U_bar) return fail(c, SDC_EINVAL, "null field pointer");
  if (parts == 0 || (parts & ~7u)) return fail(c, SDC_EINVAL, "bad parts mask");
  const Range range("rhs_vjp");
  HIPCHECK(c, hipSetDevice(c->device));
  Plan *pl;
  rc = get_plan(c, 1, box, nullptr, &pl);
  if (rc) return rc;
  const VjpLayout L = vjp_layout(pl, c->ops->ns, c->h_mech.nr, grid_cap_of(c, pl));
  const size_t need = (L.total + 64) * sizeof(double);
  if (need > c->scratch_bytes) {
    HIPCHECK(c, hipStreamSynchronize((hipStream_t)stream));
    if (c->scratch) (void)hipFree(c->scratch);
    c->scratch = nullptr;
    c->scratch_bytes = 0;
    HIPCHECK(c, hipMalloc(&c->scratch, need));
    c->scratch_bytes = need;
  }
  const LaunchCtx l = make_lc(c, pl, (hipStream_t)stream);
  rc = rhs_vjp_g(c, pl, l, U, dUdt_bar, U_bar, lnA_bar, parts, c->scratch);
  if (rc) return rc;
  HIPCHECK(c, hipGetLastError());
  return SDC_OK;
}

int set_log_prefactors(sdc_context *c, const double *lnA) {
  if (!c) return SDC_EINVAL;
  if (!c->has_mech) return fail(c, SDC_ENOMECH, "no mechanism set");
  if (!lnA && c->h_mech.nr > 0) return fail(c, SDC_EINVAL, "null lnA");
  for (int j = 0; j < c->h_mech.nr; ++j) {
    if (!std::isfinite(lnA[j])) return fail(c, SDC_EINVAL, "ln A must be finite");
    c->h_mech.lnA[j] = lnA[j];
  }
  HIPCHECK(c, hipSetDevice(c->device));
  HIPCHECK(c, hipDeviceSynchronize());
  HIPCHECK(c, hipMemcpy(c->d_mech, &c->h_mech, sizeof(DevMech), hipMemcpyHostToDevice));
  return SDC_OK;
}

int set_reference_species(sdc_context *c, int k) {
  if (!c) return SDC_EINVAL;
  if (!c->has_mech) return fail(c, SDC_ENOMECH, "no mechanism set");
  if (k < -1 || k >= c->h_mech.ns) return fail(c, SDC_EINVAL, "reference species out of range");
  if (c->h_mech.ref != k) drop_graphs(c);
  c->h_mech.ref = k;
  HIPCHECK(c, hipSetDevice(c->device));
  HIPCHECK(c, hipDeviceSynchronize());
  HIPCHECK(c, hipMemcpy(c->d_mech, &c->h_mech, sizeof(DevMech), hipMemcpyHostToDevice));
  return SDC_OK;
}

int sdc_vjp_workspace_size(const sdc_context *c, const box_desc *box, const sdc_scheme *scheme, int nsteps,
                           size_t *bytes) {
  if (!c || !bytes || nsteps < 1) return SDC_EINVAL;
  if (!c->has_mech) return SDC_ENOMECH;
  sdc_context *cc = const_cast<sdc_context *>(c);
  if (check_box(cc, box) || check_scheme(cc, scheme) || scheme->n_fine != 0 || box->nonperiodic) return SDC_EINVAL;
  Plan *pl;
  if (get_plan(cc, 1, box, nullptr, &pl)) return SDC_EHIP;
  *bytes = sdc_vjp_layout(pl, c->ops->ns, c->h_mech.nr, grid_cap_of(c, pl), scheme, nsteps).total * sizeof(double);
  return SDC_OK;
}

int sdc_step_vjp(sdc_context *c, const box_desc *box, double *U0, double dt, int nsteps,
                 const sdc_scheme *scheme, const double *UN_bar, double *U0_bar, double *lnA_bar,
                 void *workspace, size_t ws_bytes, void *stream) {
  int rc = check_vjp_args(c, box);
  if (rc) return rc;
  rc = check_scheme(c, scheme);
  if (rc) return rc;
  if (scheme->n_fine != 0) return fail(c, SDC_EINVAL, "the adjoint supports single-rate SDC (n_fine = 0)");
  if (!U0 || !UN_bar || !U0_bar) return fail(c, SDC_EINVAL, "null field pointer");
  if (nsteps < 1 || !(dt > 0)) return fail(c, SDC_EINVAL, "nsteps >= 1 and dt > 0 required");
  const Range range("sdc_step_vjp");
  HIPCHECK(c, hipSetDevice(c->device));
  Plan *pl;
  rc = get_plan(c, 1, box, nullptr, &pl);
  if (rc) return rc;
  rc = run_sdc_vjp(c, pl, U0, dt, nsteps, scheme, UN_bar, U0_bar, lnA_bar, workspace, ws_bytes,
                   (hipStream_t)stream);
  if (rc) return rc;
  HIPCHECK(c, hipGetLastError());
  return SDC_OK;
}

}  // extern "C"
