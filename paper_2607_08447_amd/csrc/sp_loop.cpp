// Host orchestration of the self-consistent Schroedinger-Poisson loop (paper
// Sec. II.B, Fig. 2a) and of the stand-alone Poisson call.  Every step runs in
// the kernels of sp.hip and the eigensolver; the host only sequences launches
// and reads back one convergence scalar per conjugate-gradient chunk and per
// loop iteration.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <string>
#include <vector>

#include "hkp_internal.h"
#include "solver.h"

#define HKP_CHECK(x)                                                              \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess)                                                         \
      throw HipError(std::string(#x) + ": " + hipGetErrorString(e_));             \
  } while (0)

namespace hkp {

namespace {

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

struct Carve {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += al(count * sizeof(T));
    return p;
  }
};

struct PoissonWS {
  double *cx, *cy, *cz, *dinv, *r, *z, *p0, *p1, *q, *partial, *n_dir;
  CGState* st;
  MGData mg;
};

// coefficients once; CG vectors and states for nrhs systems solved together; the
// multigrid levels (used unless the Jacobi preconditioner is selected)
PoissonWS carve_poisson(Carve& c, const PGeom& g, int nrhs = 1) {
  PoissonWS w;
  const long long NP = g.NP;
  const size_t nv = (size_t)nrhs * NP;
  w.cx = c.take<double>(NP);
  w.cy = c.take<double>(NP);
  w.cz = c.take<double>(NP);
  w.dinv = c.take<double>(NP);
  w.r = c.take<double>(nv);
  w.z = c.take<double>(nv);
  w.p0 = c.take<double>(nv);
  w.p1 = c.take<double>(nv);
  w.q = c.take<double>(nv);
  w.partial = c.take<double>(sp_partial_doubles(nrhs));
  w.n_dir = c.take<double>(1);
  w.st = c.take<CGState>(nrhs);
  MGData& m = w.mg;
  m.plan = mg_plan(g);
  m.ax = c.take<double>(m.plan.total);
  m.ay = c.take<double>(m.plan.total);
  m.az = c.take<double>(m.plan.total);
  m.diag = c.take<double>(m.plan.total);
  m.dinv = c.take<double>(m.plan.total);
  m.b = c.take<double>((size_t)nrhs * m.plan.vtotal);
  m.u = c.take<double>((size_t)nrhs * m.plan.vtotal);
  m.partial_rz = c.take<double>(sp_partial_doubles(nrhs));
  return w;
}

std::atomic<int> g_precond{HKP_PRECOND_MULTIGRID};

PGeom geom(const hkp_pgrid& pg) {
  return PGeom{pg.px, pg.py, pg.pz, (long long)pg.px * pg.py * pg.pz};
}

// link coefficients and preconditioner; fails without an electrode node
int poisson_prepare(const PGeom& g, double h, const double* eps, const uint8_t* dir,
                    const PoissonWS& w, hipStream_t s) {
  HKP_CHECK(launch_pcoef(g, h, eps, dir, w.cx, w.cy, w.cz, w.dinv, w.partial, w.n_dir, s));
  double nd = 0.0;
  HKP_CHECK(hipMemcpyAsync(&nd, w.n_dir, sizeof(double), hipMemcpyDeviceToHost, s));
  HKP_CHECK(hipStreamSynchronize(s));
  if (!(nd > 0.0)) {
    set_error("the Poisson box has no electrode (Dirichlet) node");
    return HKP_E_ARG;
  }
  if (g_precond.load() == HKP_PRECOND_MULTIGRID)
    HKP_CHECK(launch_mg_setup(g, w.cx, w.cy, w.cz, dir, w.mg, s));
  return HKP_OK;
}

// A chunk of CG iterations recorded once as a hipGraph (kernels only) and
// replayed: the launches of one iteration are short, so their gaps matter.
// Reused while everything the recorded launches take stays the same: the
// solution, electrode-mask and workspace buffers, the box, the iteration cap, the
// number of systems, the preconditioner and the device.
struct CGGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const double* phi = nullptr;
  const uint8_t* dir = nullptr;
  const void* ws = nullptr;
  int px = 0, py = 0, pz = 0;
  int max_iter = -1;
  int nrhs = 0;
  int precond = -1;
  int device = -1;
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~CGGraph() { reset(); }
};

// iterations per chunk, even (every chunk starts from the same direction buffer): a
// multigrid-preconditioned solve needs tens of iterations, a Jacobi one hundreds
int cg_chunk(bool mg) { return mg ? 8 : 32; }

void launch_cg_chunk(const PGeom& g, const uint8_t* dir, double* phi, int max_iter,
                     const PoissonWS& w, hipStream_t s, int nrhs, bool mg) {
  for (int c = 0; c < cg_chunk(mg); ++c) {
    double* po = (c % 2 == 0) ? w.p0 : w.p1;
    double* pn = (c % 2 == 0) ? w.p1 : w.p0;
    // with multigrid r and z trade buffers every iteration (chunks are even)
    double* z = (mg && c % 2 == 1) ? w.r : w.z;
    double* r = (mg && c % 2 == 1) ? w.z : w.r;
    HKP_CHECK(launch_cg_iter(g, w.cx, w.cy, w.cz, w.dinv, dir, z, po, pn, w.q, phi, r,
                             w.partial, max_iter, w.st, s, nrhs, mg ? &w.mg : nullptr));
  }
}

// conjugate gradients from the guess in phi; launches run in chunks (recorded as
// a graph when the stream can be captured), the host reads the device state once
// per chunk (iterations after convergence are no-ops)
int poisson_cg(const PGeom& g, const uint8_t* dir, const double* phi_fixed, const double* rho,
               double* phi, double tol, int max_iter, const PoissonWS& w, hipStream_t s,
               int* iters, double* relres, CGGraph* gc = nullptr, int nrhs = 1) {
  const int precond = g_precond.load();
  const bool mg = precond == HKP_PRECOND_MULTIGRID;
  HKP_CHECK(launch_cg_init(g, w.cx, w.cy, w.cz, w.dinv, dir, phi_fixed, rho, kEoverEps0, phi,
                           w.r, w.z, w.p0, w.partial, tol, w.st, s, nrhs));
  if (mg) HKP_CHECK(launch_mg_start(g, w.mg, w.r, w.z, w.st, nrhs, s));
  int device = -1;
  HKP_CHECK(hipGetDevice(&device));
  if (gc && s != nullptr &&
      (gc->phi != phi || gc->dir != dir || gc->ws != w.st || gc->px != g.px || gc->py != g.py ||
       gc->pz != g.pz || gc->max_iter != max_iter || gc->nrhs != nrhs ||
       gc->precond != precond || gc->device != device || !gc->exec)) {
    gc->reset();
    HKP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
      launch_cg_chunk(g, dir, phi, max_iter, w, s, nrhs, mg);
    } catch (...) {
      hipGraph_t g2 = nullptr;
      (void)hipStreamEndCapture(s, &g2);
      if (g2) (void)hipGraphDestroy(g2);
      throw;
    }
    HKP_CHECK(hipStreamEndCapture(s, &gc->graph));
    HKP_CHECK(hipGraphInstantiate(&gc->exec, gc->graph, nullptr, nullptr, 0));
    gc->phi = phi;
    gc->dir = dir;
    gc->ws = w.st;
    gc->px = g.px;
    gc->py = g.py;
    gc->pz = g.pz;
    gc->max_iter = max_iter;
    gc->nrhs = nrhs;
    gc->precond = precond;
    gc->device = device;
  }
  const bool use_graph = gc && s != nullptr && gc->exec;
  std::vector<CGState> h((size_t)nrhs);
  long long launched = 0;
  for (;;) {
    HKP_CHECK(hipMemcpyAsync(h.data(), w.st, sizeof(CGState) * nrhs, hipMemcpyDeviceToHost, s));
    HKP_CHECK(hipStreamSynchronize(s));
    bool all = true;
    for (const CGState& x : h) all = all && x.done;
    if (all || launched >= max_iter) break;
    if (use_graph)
      HKP_CHECK(hipGraphLaunch(gc->exec, s));
    else
      launch_cg_chunk(g, dir, phi, max_iter, w, s, nrhs, mg);
    launched += cg_chunk(mg);
  }
  // the worst system: most iterations, largest relative residual
  int it = 0, rc = HKP_OK;
  double rel = 0.0;
  for (const CGState& x : h) {
    it = std::max(it, x.it);
    rel = std::max(rel, x.bb > 0.0 ? std::sqrt(x.rr / x.bb) : 0.0);
    if (x.breakdown) {
      set_error("Poisson CG breakdown: the operator is not positive definite (a free region "
                "without a path to an electrode?)");
      return HKP_E_NUMERICAL;
    }
    if (!(x.rr <= x.thr)) rc = HKP_W_NOT_CONVERGED;
  }
  if (iters) *iters = it;
  if (relres) *relres = rel;
  return rc;
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

int set_poisson_precond(int kind) { return g_precond.exchange(kind); }

size_t poisson_bytes(const hkp_pgrid& pg) {
  Carve c{nullptr};
  carve_poisson(c, geom(pg));
  return c.off;
}

int run_poisson(const PoissonArgs& a, int* iters, double* relres) {
  const PGeom g = geom(a.pg);
  hipStream_t s = reinterpret_cast<hipStream_t>(a.stream);
  Carve c{reinterpret_cast<char*>(a.workspace)};
  const PoissonWS w = carve_poisson(c, g);
  const int rc = poisson_prepare(g, a.h, a.eps, a.dir, w, s);
  if (rc != HKP_OK) return rc;
  // one recorded chunk per host thread, kept across calls (repeated solves with the
  // same buffers skip recording); never destroyed, so nothing runs at process exit
  // after the HIP runtime has gone
  thread_local CGGraph* gc = new CGGraph;
  return poisson_cg(g, a.dir, a.phi_fixed, a.rho, a.phi, a.tol, a.max_iter, w, s, iters,
                    relres, gc);
}

namespace {

struct SPLayout {
  size_t solver;   // eigensolver workspace (first, at offset 0)
  double2* block;  // [nb][nx][ny][nz][6] ABI spinors: restart block and psi
  double *V, *Vref, *dV, *eig, *resid, *f, *mu;
  PoissonWS pw;
  double *phi_out, *rho, *F, *histX, *histF, *G, *dots, *gamma, *delta;
  size_t total;
};

SPLayout carve_sp(char* base, const Plan& p, const hkp_pgrid& pg, int m) {
  SPLayout L;
  Carve c{base};
  L.solver = al(plan_bytes(p));
  c.off = L.solver;
  const long long NP = geom(pg).NP;
  L.block = c.take<double2>((size_t)p.nb * p.n6);
  L.V = c.take<double>(p.N);
  L.Vref = c.take<double>(p.N);
  L.dV = c.take<double>(1);
  L.eig = c.take<double>(p.nb);
  L.resid = c.take<double>(p.nb);
  L.f = c.take<double>(p.nb);
  L.mu = c.take<double>(1);
  L.pw = carve_poisson(c, geom(pg));
  L.phi_out = c.take<double>(NP);
  L.rho = c.take<double>(NP);
  L.F = c.take<double>(NP);
  L.histX = c.take<double>((size_t)std::max(m, 1) * NP);
  L.histF = c.take<double>((size_t)std::max(m, 1) * NP);
  L.G = c.take<double>(64);
  L.dots = c.take<double>(16);
  L.gamma = c.take<double>(8);
  L.delta = c.take<double>(1);
  L.total = c.off;
  return L;
}

}  // namespace

size_t sp_bytes(const hkp_grid& g, const hkp_opts& o, const hkp_pgrid& pg,
                const hkp_sp_opts& sp) {
  return carve_sp(nullptr, make_plan(g, o, 1), pg, sp.history).total;
}

int run_sp(const SPArgs& a, hkp_sp_stats* stats) {
  const auto t_start = std::chrono::steady_clock::now();
  hipStream_t s = reinterpret_cast<hipStream_t>(a.stream);
  const Plan p = make_plan(a.grid, a.opts, 1);
  const PGeom g = geom(a.pg);
  const int m = a.sp.history;
  char* base = reinterpret_cast<char*>(a.workspace);
  const SPLayout L = carve_sp(base, p, a.pg, m);
  const int ox = a.pg.ox, oy = a.pg.oy, oz = a.pg.oz;
  const double h = a.grid.h_nm;

  hkp_sp_stats st{};
  st.solve_status = HKP_OK;
  st.f_last = 0.0;
  double t_sch = 0.0, t_poi = 0.0;

  int rc = poisson_prepare(g, h, a.eps, a.dir, L.pw, s);
  if (rc != HKP_OK) return rc;
  CGGraph cg_graph;
  // the fixed charge alone (the hole part of rho is added every iteration)
  HKP_CHECK(launch_rho(g, ox, oy, oz, p.nx, p.ny, p.nz, 0, nullptr, 0, nullptr, 0.0,
                       a.rho_fixed, L.rho, nullptr, s));
  if (!(a.sp.flags & HKP_SP_PHI0)) {
    // start from the hole-free potential
    HKP_CHECK(hipMemsetAsync(a.phi, 0, (size_t)g.NP * sizeof(double), s));
    int it = 0;
    const auto t0 = std::chrono::steady_clock::now();
    rc = poisson_cg(g, a.dir, a.phi_fixed, L.rho, a.phi, a.sp.cg_tol, a.sp.cg_max_iter, L.pw, s,
                    &it, nullptr, &cg_graph);
    t_poi += seconds_since(t0);
    st.cg_iters += it;
    if (rc < 0) return rc;
  } else {
    // the caller's potential, with the electrode values imposed
    HKP_CHECK(launch_cg_init(g, L.pw.cx, L.pw.cy, L.pw.cz, L.pw.dinv, a.dir, a.phi_fixed, L.rho,
                             kEoverEps0, a.phi, L.pw.r, L.pw.z, L.pw.p0, L.pw.partial, 1.0,
                             L.pw.st, s));
  }

  SolveArgs sa{};
  sa.plan = p;
  sa.mat = a.mat;
  sa.V = L.V;
  sa.strain = a.strain;
  for (int i = 0; i < 3; ++i) sa.B[i] = a.B[i];
  sa.eig = L.eig;
  sa.psi = L.block;
  sa.resid = L.resid;
  sa.workspace = base;
  sa.stream = a.stream;
  sa.tol = a.opts.tol_eV;
  sa.max_iter = a.opts.max_iter;
  sa.seed = a.opts.seed;
  sa.st = autotuned(a.grid, p.nb, p.mixed, stencil_variant(a.strain != nullptr, a.B));
  sa.graph_chunk = 4;
  const int base_flags = (a.opts.flags & ~(HKP_FLAG_X0 | HKP_FLAG_X0_NEV)) | HKP_FLAG_PSI_BLOCK;

  // annealing: the loop first runs at anneal_K, where the thermal spread of the
  // occupations exceeds the small level splittings near the Fermi level and the
  // density answers the potential smoothly; once that stage is within 1 mV of
  // its fixed point the loop goes on at the requested temperature (same
  // potential, eigenvector block and bound; the Anderson history is cleared)
  bool annealing = a.sp.anneal_K > a.sp.temperature_K;
  double kT = kBoltzmann * (annealing ? a.sp.anneal_K : a.sp.temperature_K);
  // the annealing stage only has to reach the basin of the final fixed point
  const double anneal_tol = std::max(a.sp.tol_V, 1e-3);
  const bool adaptive = !(a.sp.flags & HKP_SP_EXACT_EIG);
  int count = 0;   // entries pushed into the Anderson history
  bool converged = false, final_pass = false;
  // a caller's starting potential may already be converged: its first
  // eigensolve goes to opts->tol (from the hole-free start, to 1e-4 eV)
  double delta = 0.0, delta_prev = (a.sp.flags & HKP_SP_PHI0) ? 0.0 : HUGE_VAL;
  int it = 0;
  double bound = 0.0;   // the Lanczos upper spectral bound of H(V_ref)
  // HKP_SP_TRACE=1 prints one line per iteration to stderr (diagnostics)
  const char* tr = std::getenv("HKP_SP_TRACE");
  const bool trace = tr && tr[0] == '1';
  for (it = 1; it <= a.sp.max_iter; ++it) {
    // Schroedinger: V = V_off + phi on the embedded grid; restart from the last block.
    // Eigensolves stop at a residual tied to how far the potential still moves
    // (an eigenvector error of r / gap moves the Hartree potential far less than
    // the loop's own step while r <= 0.01 delta); the final pass uses opts->tol.
    auto t0 = std::chrono::steady_clock::now();
    HKP_CHECK(launch_extract(p.nx, p.ny, p.nz, g, ox, oy, oz, a.V_off, a.phi, L.V, s));
    // only V changes between iterations: by Weyl's inequality the upper bound of the
    // spectrum that the first solve's Lanczos run found, plus max |V - V_ref| (V_ref
    // that solve's potential), bounds the new one; no Lanczos run after the first.
    // (Adding each step's change to the last bound instead would grow with the path
    // the loop takes, not with its distance from V_ref, and loosen the filter.)
    sa.bound_hint = 0.0;
    if (it > 1 && bound > 0.0) {
      const PGeom gv{p.nx, p.ny, p.nz, p.N};   // elementwise over the Schroedinger grid
      HKP_CHECK(launch_residual_max(gv, L.Vref, L.V, L.F, L.pw.partial, L.dV, s));
      double dv = 0.0;
      HKP_CHECK(hipMemcpyAsync(&dv, L.dV, sizeof(double), hipMemcpyDeviceToHost, s));
      HKP_CHECK(hipStreamSynchronize(s));
      if (std::isfinite(dv)) sa.bound_hint = bound + dv;
    }
    sa.X0 = it > 1 ? L.block : nullptr;
    sa.flags = base_flags | (it > 1 ? HKP_FLAG_X0 : 0);
    sa.tol = (adaptive && !final_pass)
                 ? std::max(a.opts.tol_eV, std::min(1e-4, 0.01 * delta_prev))
                 : a.opts.tol_eV;
    hkp_stats sst{};
    rc = run_solve(sa, &sst);
    if (rc < 0) return rc;
    if (rc != HKP_OK) st.solve_status = rc;
    st.schroedinger_iters += sst.iters;
    if (sa.bound_hint == 0.0) {   // a Lanczos bound: the new reference
      bound = sst.lambda_max_bound;
      HKP_CHECK(hipMemcpyAsync(L.Vref, L.V, (size_t)p.N * sizeof(double),
                               hipMemcpyDeviceToDevice, s));
    }
    t_sch += seconds_since(t0);

    // occupancy, hole density, Poisson from the current potential
    t0 = std::chrono::steady_clock::now();
    HKP_CHECK(launch_occupancy(p.nev, L.eig, a.sp.n_holes, kT, L.f, L.mu, s));
    HKP_CHECK(launch_rho(g, ox, oy, oz, p.nx, p.ny, p.nz, p.nev, L.block, p.n6, L.f,
                         1.0 / (h * h * h), a.rho_fixed, L.rho, nullptr, s));
    HKP_CHECK(hipMemcpyAsync(L.phi_out, a.phi, (size_t)g.NP * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    int cgit = 0;
    // the Poisson solve, like the eigensolve, need not be tighter than the
    // loop's own step until the final pass
    const double cg_tol = (adaptive && !final_pass)
                              ? std::max(a.sp.cg_tol, std::min(1e-6, 1e-2 * delta_prev))
                              : a.sp.cg_tol;
    rc = poisson_cg(g, a.dir, a.phi_fixed, L.rho, L.phi_out, cg_tol, a.sp.cg_max_iter, L.pw, s,
                    &cgit, nullptr, &cg_graph);
    st.cg_iters += cgit;
    if (rc < 0) return rc;
    if (rc != HKP_OK) st.poisson_status = rc;
    HKP_CHECK(launch_residual_max(g, a.phi, L.phi_out, L.F, L.pw.partial, L.delta, s));
    HKP_CHECK(hipMemcpyAsync(&delta, L.delta, sizeof(double), hipMemcpyDeviceToHost, s));
    HKP_CHECK(hipStreamSynchronize(s));
    t_poi += seconds_since(t0);
    if (!std::isfinite(delta)) {
      set_error("self-consistent loop diverged (non-finite potential update)");
      return HKP_E_NUMERICAL;
    }
    if (trace)
      std::fprintf(stderr, "[hkp sp] it %d  max|F| %.3e V  eig tol %.1e (%d iters)  cg tol %.1e "
                   "(%d iters)  history %d%s\n", it, delta, sa.tol, sst.iters, cg_tol, cgit,
                   std::min(count, m), annealing ? "  (annealing)" : "");
    if (annealing) {
      if (delta <= anneal_tol) {
        // the next iteration evaluates the same potential at the requested temperature
        annealing = false;
        kT = kBoltzmann * a.sp.temperature_K;
        st.anneal_iters = it;
        count = 0;
        delta_prev = delta;
        continue;
      }
    } else if (delta <= a.sp.tol_V) {
      if (sa.tol <= a.opts.tol_eV && cg_tol <= a.sp.cg_tol) {
        converged = true;
        break;
      }
      // met with a looser eigensolve: one more pass at this potential and opts->tol
      final_pass = true;
      continue;
    }
    final_pass = false;
    delta_prev = delta;
    if (it == a.sp.max_iter) break;
    // next input potential
    const int k = std::min(count, m);
    const int slot = m > 0 ? count % m : -1;
    HKP_CHECK(launch_anderson(g, k, m, slot, a.sp.mixing, a.phi, L.F, L.histX, L.histF, L.G,
                              L.dots, L.gamma, L.pw.partial, s));
    ++count;
  }
  if (it > a.sp.max_iter) it = a.sp.max_iter;

  // outputs: the eigenpairs and density of the last input potential
  HKP_CHECK(hipMemcpyAsync(a.eig, L.eig, (size_t)p.nev * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
  if (a.resid)
    HKP_CHECK(hipMemcpyAsync(a.resid, L.resid, (size_t)p.nev * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
  if (a.psi)
    HKP_CHECK(hipMemcpyAsync(a.psi, L.block, (size_t)p.nev * p.n6 * sizeof(double2),
                             hipMemcpyDeviceToDevice, s));
  if (a.density)
    HKP_CHECK(launch_rho(g, ox, oy, oz, p.nx, p.ny, p.nz, p.nev, L.block, p.n6, L.f,
                         1.0 / (h * h * h), nullptr, nullptr, a.density, s));
  double mu = 0.0;
  double flast = 0.0;
  HKP_CHECK(hipMemcpyAsync(&mu, L.mu, sizeof(double), hipMemcpyDeviceToHost, s));
  HKP_CHECK(hipMemcpyAsync(&flast, L.f + (p.nev - 1), sizeof(double), hipMemcpyDeviceToHost, s));
  HKP_CHECK(hipStreamSynchronize(s));

  st.iters = it;
  if (annealing) st.anneal_iters = it;   // never left the annealing temperature
  st.converged = converged ? 1 : 0;
  st.delta_V = delta;
  st.mu_eV = mu;
  st.f_last = flast;
  st.nb = p.nb;
  st.seconds = seconds_since(t_start);
  st.t_schroedinger = t_sch;
  st.t_poisson = t_poi;
  if (stats) *stats = st;
  if (!converged) return HKP_W_NOT_CONVERGED;
  return st.solve_status != HKP_OK ? st.solve_status : HKP_OK;
}

namespace {

struct CILayout {
  PoissonWS pw;
  double *rhs, *V, *comp, *gpart, *hsp, *A, *Vc, *Cs, *H, *vecs, *evals;
  int* status;
  size_t total;
};

CILayout carve_ci(char* base, const hkp_grid& g, int M, const hkp_pgrid& pg) {
  CILayout L;
  Carve c{base};
  const long long NP = geom(pg).NP, NS = (long long)g.nx * g.ny * g.nz;
  const int P = M * (M + 1) / 2, K = M * (2 * M - 1);
  L.pw = carve_poisson(c, geom(pg), 2 * P);
  L.rhs = c.take<double>((size_t)2 * P * NP);
  L.V = c.take<double>((size_t)2 * P * NP);
  L.comp = c.take<double>((size_t)2 * 3 * M * NS);
  const int wide = std::max(std::max(3 * M, M * M), P);
  L.gpart = c.take<double>(gram_partial_bytes(wide, NS, 1) / sizeof(double));
  L.hsp = c.take<double>((size_t)2 * 4 * M * M);
  L.A = c.take<double>((size_t)2 * M * M * NS);
  L.Vc = c.take<double>((size_t)2 * P * NS);
  L.Cs = c.take<double>((size_t)2 * M * M * P);
  L.H = c.take<double>((size_t)2 * K * K);
  L.vecs = c.take<double>((size_t)2 * K * K);
  L.evals = c.take<double>(K);
  L.status = c.take<int>(1);
  L.total = c.off;
  return L;
}

}  // namespace

size_t ci_bytes(const hkp_grid& g, int M, const hkp_pgrid& pg) {
  return carve_ci(nullptr, g, M, pg).total;
}

int run_ci(const CIArgs& a, hkp_ci_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = reinterpret_cast<hipStream_t>(a.stream);
  const CILayout L = carve_ci(reinterpret_cast<char*>(a.workspace), a.grid, a.M, a.pg);
  const PGeom g = geom(a.pg);
  const int M = a.M, P = M * (M + 1) / 2, K = M * (2 * M - 1), nrhs = 2 * P;
  const long long NS = (long long)a.grid.nx * a.grid.ny * a.grid.nz;
  const int nx = a.grid.nx, ny = a.grid.ny, nz = a.grid.nz;
  // single-particle matrix diag(E) (x) 1 + spin-orbit (component overlaps on the Gram kernel)
  HKP_CHECK(launch_gather_components(NS, M, a.phi, L.comp, s));
  const BlockDesc Bc{L.comp, NS, 3 * M, 3LL * M * NS};
  HKP_CHECK(launch_gram(Bc, Bc, 1, 1, L.gpart, L.A, nullptr, s));   // overlaps into A (scratch)
  HKP_CHECK(launch_soi_assemble(M, L.A, a.E, a.delta_so, L.hsp, s));
  // pair densities -> potentials with every electrode grounded, all pairs at once
  int rc = poisson_prepare(g, a.grid.h_nm, a.eps, a.dir, L.pw, s);
  if (rc != HKP_OK) return rc;
  HKP_CHECK(launch_pair_rhs(g, a.pg.ox, a.pg.oy, a.pg.oz, nx, ny, nz, M, a.phi, a.grid.h_nm,
                            L.rhs, s));
  HKP_CHECK(hipMemsetAsync(L.V, 0, (size_t)nrhs * g.NP * sizeof(double), s));
  const auto tp = std::chrono::steady_clock::now();
  int cgit = 0;
  double rel = 0.0;
  CGGraph gc;
  rc = poisson_cg(g, a.dir, nullptr, L.rhs, L.V, a.cg_tol, a.cg_max_iter, L.pw, s, &cgit, &rel,
                  &gc, nrhs);
  const double t_poisson =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - tp).count();
  if (rc < 0) return rc;
  const int poisson_status = rc;
  // Coulomb integrals (ik|jl) = sum over the grid of conj(A_ik) V_jl (Gram kernel)
  HKP_CHECK(launch_pair_potential_gather(g, a.pg.ox, a.pg.oy, a.pg.oz, nx, ny, nz, P, L.V, L.Vc,
                                         s));
  HKP_CHECK(launch_pair_product(NS, M, a.phi, L.A, s));
  const BlockDesc BA{L.A, NS, M * M, (long long)M * M * NS};
  const BlockDesc BV{L.Vc, NS, P, (long long)P * NS};
  HKP_CHECK(launch_gram(BA, BV, 0, 1, L.gpart, L.Cs, nullptr, s));
  // determinant matrix, its spectrum, the exchange splitting
  HKP_CHECK(launch_ci_assemble(M, L.hsp, L.Cs, L.H, s));
  if (a.H)
    HKP_CHECK(hipMemcpyAsync(a.H, L.H, (size_t)K * K * 16, hipMemcpyDeviceToDevice, s));
  if (a.coulomb)
    HKP_CHECK(launch_coulomb_expand(M, L.Cs, static_cast<double*>(a.coulomb), s));
  HKP_CHECK(hipMemsetAsync(L.status, 0, sizeof(int), s));
  HKP_CHECK(launch_heev(L.H, K, 1, (long long)K * K, a.eig,
                        a.vecs ? static_cast<double*>(a.vecs) : L.vecs, 0, L.status, nullptr, s));
  if (a.J && K >= 4) HKP_CHECK(launch_exchange(a.eig, a.J, s));
  HKP_CHECK(hipStreamSynchronize(s));
  if (stats) {
    stats->cg_iters = cgit;
    stats->cg_relres = rel;
    stats->poisson_solves = nrhs - M;   // the diagonal pairs' imaginary parts are zero
    stats->determinants = K;
    stats->t_poisson = t_poisson;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return poisson_status;
}

}  // namespace hkp
