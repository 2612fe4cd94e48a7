// C ABI entry points (include/hkp.h): argument validation, workspace checks
// and translation of failures into return codes.  No exception crosses the
// ABI; nothing is enqueued on the GPU before the arguments have been checked.
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "hkp_internal.h"
#include "solver.h"

namespace hkp {

namespace {
thread_local std::string g_err = "no error";

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int check_grid(const hkp_grid* g) {
  if (!g) {
    set_error("grid is NULL");
    return HKP_E_ARG;
  }
  if (g->nx < 1 || g->ny < 1 || g->nz < 1 || !finite_pos(g->h_nm)) {
    set_error("grid needs nx, ny, nz >= 1 and h > 0");
    return HKP_E_ARG;
  }
  const long long N = (long long)g->nx * g->ny * g->nz;
  if (N > (1LL << 31) / 6) {
    set_error("grid too large");
    return HKP_E_ARG;
  }
  return HKP_OK;
}

int check_material(const hkp_material* m) {
  if (!m) {
    set_error("material is NULL");
    return HKP_E_ARG;
  }
  const double v[] = {m->gamma1, m->gamma2, m->gamma3, m->delta_so_eV,
                      m->kappa,  m->a_v_eV, m->b_eV,   m->d_eV};
  for (double x : v)
    if (!std::isfinite(x)) {
      set_error("material parameter is not finite");
      return HKP_E_ARG;
    }
  return HKP_OK;
}

int check_field(const double* B) {
  if (!B) {
    set_error("B_T is NULL");
    return HKP_E_ARG;
  }
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(B[i])) {
      set_error("B is not finite");
      return HKP_E_ARG;
    }
  return HKP_OK;
}

int check_opts(const hkp_grid* g, const hkp_opts* o) {
  if (!o) {
    set_error("opts is NULL");
    return HKP_E_ARG;
  }
  // unknowns per vector: 6 N, or 3 N for the spin-free orbital problem
  const long long n6 = ((o->flags & HKP_FLAG_SPIN_FREE) ? 3LL : 6LL) * g->nx * g->ny * g->nz;
  if (o->nev < 1 || o->nev > n6) {
    set_error("nev must satisfy 1 <= nev <= 6 N (3 N spin-free)");
    return HKP_E_ARG;
  }
  const int nb = block_size(*g, *o);
  if (o->nb < 0 || nb > HKP_NB_MAX || nb > n6 || nb <= o->nev) {
    set_error("block size must satisfy nev < nb <= min(64, 6 N) (3 N spin-free)");
    return HKP_E_ARG;
  }
  if (o->degree < 0 || o->degree > 200) {
    set_error("degree must be 0 (default schedule) or 1..200");
    return HKP_E_ARG;
  }
  if (o->max_iter < 1) {
    set_error("max_iter must be >= 1");
    return HKP_E_ARG;
  }
  if (!(o->tol_eV > 0.0) || !std::isfinite(o->tol_eV)) {
    set_error("tol must be > 0");
    return HKP_E_ARG;
  }
  if (o->precision != HKP_PREC_FP64 && o->precision != HKP_PREC_MIXED) {
    set_error("precision must be HKP_PREC_FP64 or HKP_PREC_MIXED");
    return HKP_E_ARG;
  }
  return HKP_OK;
}

// The current device must be a gfx950.  The architecture check reads the device
// properties, which takes milliseconds; a device found to be a gfx950 is
// remembered (per device index), so later calls only ask for the current device.
constexpr int kMaxDevices = 64;
std::atomic<bool> g_device_ok[kMaxDevices] = {};

int check_device() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_error(std::string("no HIP device: ") + hipGetErrorString(e));
    return HKP_E_UNSUPPORTED;
  }
  if (dev >= 0 && dev < kMaxDevices && g_device_ok[dev].load(std::memory_order_relaxed))
    return HKP_OK;
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) {
    set_error(std::string("hipGetDeviceProperties: ") + hipGetErrorString(e));
    return HKP_E_HIP;
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    set_error(std::string("unsupported GPU architecture ") + prop.gcnArchName +
              " (built for gfx950)");
    return HKP_E_UNSUPPORTED;
  }
  if (dev >= 0 && dev < kMaxDevices) g_device_ok[dev].store(true, std::memory_order_relaxed);
  return HKP_OK;
}

int check_pgrid(const hkp_pgrid* pg, const hkp_grid* g) {
  if (!pg) {
    set_error("pgrid is NULL");
    return HKP_E_ARG;
  }
  if (pg->px < 1 || pg->py < 1 || pg->pz < 1) {
    set_error("Poisson box needs px, py, pz >= 1");
    return HKP_E_ARG;
  }
  if ((long long)pg->px * pg->py * pg->pz > (1LL << 31)) {
    set_error("Poisson box too large");
    return HKP_E_ARG;
  }
  if (g && (pg->ox < 0 || pg->oy < 0 || pg->oz < 0 || pg->ox + g->nx > pg->px ||
            pg->oy + g->ny > pg->py || pg->oz + g->nz > pg->pz)) {
    set_error("the Schroedinger grid must lie inside the Poisson box");
    return HKP_E_ARG;
  }
  return HKP_OK;
}

int check_sp_opts(const hkp_sp_opts* sp, int nev) {
  if (!sp) {
    set_error("sp opts is NULL");
    return HKP_E_ARG;
  }
  if (!(sp->n_holes >= 0.0 && sp->n_holes <= nev)) {
    set_error("n_holes must satisfy 0 <= n_holes <= nev");
    return HKP_E_ARG;
  }
  if (!finite_pos(sp->temperature_K) || !(sp->mixing > 0.0 && sp->mixing <= 1.0) ||
      sp->history < 0 || sp->history > 8 || sp->max_iter < 1 || !finite_pos(sp->tol_V) ||
      !finite_pos(sp->cg_tol) || sp->cg_max_iter < 1 ||
      !(std::isfinite(sp->anneal_K) && sp->anneal_K >= 0.0)) {
    set_error("sp opts: T > 0, 0 < mixing <= 1, history 0..8, max_iter >= 1, tol_V > 0, "
              "cg_tol > 0, cg_max_iter >= 1, finite anneal_K >= 0");
    return HKP_E_ARG;
  }
  return HKP_OK;
}

#define HKP_TRY(x)            \
  do {                        \
    int r_ = (x);             \
    if (r_ != HKP_OK) return r_; \
  } while (0)

int solve_common(const hkp_grid* grid, const hkp_material* mat, const hkp_opts* opts,
                 int32_t batch, const double* V, const double* strain, const double B[3],
                 const void* X0, double* eig, void* psi, double* resid, void* ws,
                 size_t ws_bytes, void* stream, hkp_stats* stats) {
  HKP_TRY(check_grid(grid));
  HKP_TRY(check_material(mat));
  HKP_TRY(check_field(B));
  HKP_TRY(check_opts(grid, opts));
  if (batch < 1 || batch > 65535) {
    set_error("batch must be in 1..65535");
    return HKP_E_ARG;
  }
  if (!V || !eig || !ws) {
    set_error("V, eig_eV and workspace must not be NULL");
    return HKP_E_ARG;
  }
  if ((opts->flags & HKP_FLAG_X0) && !X0) {
    set_error("HKP_FLAG_X0 needs X0");
    return HKP_E_ARG;
  }
  if ((opts->flags & HKP_FLAG_GRAPH) && stream == nullptr) {
    set_error("HKP_FLAG_GRAPH needs a non-default stream (the legacy stream cannot be captured)");
    return HKP_E_ARG;
  }
  if ((opts->flags & HKP_FLAG_SPIN_FREE) && (B[0] != 0.0 || B[1] != 0.0 || B[2] != 0.0)) {
    set_error("HKP_FLAG_SPIN_FREE needs B = 0");
    return HKP_E_ARG;
  }
  Plan p = make_plan(*grid, *opts, batch);
  const size_t need = plan_bytes(p);
  if (ws_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return HKP_E_WORKSPACE;
  }
  HKP_TRY(check_device());
  SolveArgs a{};
  a.plan = p;
  a.mat = *mat;
  if (opts->flags & HKP_FLAG_SPIN_FREE) a.mat.delta_so_eV = 0.0;   // H_0 has no spin-orbit term
  a.V = V;
  a.strain = strain;
  for (int i = 0; i < 3; ++i) a.B[i] = B[i];
  a.X0 = (opts->flags & HKP_FLAG_X0) ? X0 : nullptr;
  a.eig = eig;
  a.psi = psi;
  a.resid = resid;
  a.workspace = ws;
  a.stream = stream;
  a.tol = opts->tol_eV;
  a.max_iter = opts->max_iter;
  a.flags = opts->flags;
  a.seed = opts->seed;
  a.st = autotuned(*grid, p.nb, p.mixed, stencil_variant(strain != nullptr, B));
  a.graph_chunk = 4;
  return guarded([&]() { return run_solve(a, stats); });
}

}  // namespace

void set_error(const std::string& msg) { g_err = msg; }

}  // namespace hkp

using namespace hkp;

extern "C" {

void hkp_default_material(hkp_material* m) {
  if (!m) return;
  m->gamma1 = 4.285;
  m->gamma2 = 0.339;
  m->gamma3 = 1.446;
  m->delta_so_eV = 0.044;
  m->kappa = -0.42;
  m->a_v_eV = 2.46;
  m->b_eV = -2.35;
  m->d_eV = -5.32;
}

void hkp_unit_constants(double out[3]) {
  if (!out) return;
  out[0] = kE0;
  out[1] = kMuB;
  out[2] = kEoverHbar;
}

void hkp_default_opts(hkp_opts* o) {
  if (!o) return;
  o->nev = 8;
  o->nb = 0;
  o->degree = 0;
  o->max_iter = 200;
  o->tol_eV = 1e-8;
  o->precision = HKP_PREC_FP64;
  o->flags = 0;
  o->seed = 1;
}

int32_t hkp_block_size(const hkp_grid* grid, const hkp_opts* opts) {
  if (check_grid(grid) != HKP_OK || check_opts(grid, opts) != HKP_OK) return 0;
  return block_size(*grid, *opts);
}

size_t hkp_workspace_bytes(const hkp_grid* grid, const hkp_opts* opts, int32_t batch) {
  if (check_grid(grid) != HKP_OK || check_opts(grid, opts) != HKP_OK) return 0;
  if (batch < 1 || batch > 65535) {
    set_error("batch must be in 1..65535");
    return 0;
  }
  return plan_bytes(make_plan(*grid, *opts, batch));
}

int hkp_solve(const hkp_grid* grid, const hkp_material* mat, const hkp_opts* opts,
              const double* V_eV, const double* strain, const double B_T[3], const void* X0,
              double* eig_eV, void* psi, double* resid_eV, void* workspace, size_t ws_bytes,
              void* hip_stream, hkp_stats* stats) {
  return solve_common(grid, mat, opts, 1, V_eV, strain, B_T, X0, eig_eV, psi, resid_eV,
                      workspace, ws_bytes, hip_stream, stats);
}

int hkp_solve_batch(const hkp_grid* grid, const hkp_material* mat, const hkp_opts* opts,
                    int32_t batch, const double* V_eV, const double* strain, const double B_T[3],
                    const void* X0, double* eig_eV, void* psi, double* resid_eV,
                    void* workspace, size_t ws_bytes, void* hip_stream, hkp_stats* stats) {
  return solve_common(grid, mat, opts, batch, V_eV, strain, B_T, X0, eig_eV, psi, resid_eV,
                      workspace, ws_bytes, hip_stream, stats);
}

size_t hkp_apply_workspace_bytes(const hkp_grid* grid, int32_t nvec) {
  if (check_grid(grid) != HKP_OK) return 0;
  if (nvec < 1) {
    set_error("nvec must be >= 1");
    return 0;
  }
  return apply_bytes(*grid, nvec);
}

int hkp_filter_step(const hkp_grid* grid, const hkp_material* mat, const double* V_eV,
                    const double* strain, const double B_T[3], int32_t nvec, const void* X,
                    const void* Y_old, void* Y, double alpha, double shift, double beta,
                    int32_t precision, void* workspace, size_t ws_bytes, void* hip_stream) {
  HKP_TRY(check_grid(grid));
  HKP_TRY(check_material(mat));
  HKP_TRY(check_field(B_T));
  if (nvec < 1 || !V_eV || !X || !Y || !workspace) {
    set_error("nvec >= 1 and non-NULL V, X, Y, workspace required");
    return HKP_E_ARG;
  }
  if (!std::isfinite(alpha) || !std::isfinite(shift) || !std::isfinite(beta)) {
    set_error("alpha, shift, beta must be finite");
    return HKP_E_ARG;
  }
  if (beta != 0.0 && !Y_old) {
    set_error("beta != 0 needs Y_old");
    return HKP_E_ARG;
  }
  if (precision != HKP_PREC_FP64 && precision != HKP_PREC_MIXED) {
    set_error("precision must be HKP_PREC_FP64 or HKP_PREC_MIXED");
    return HKP_E_ARG;
  }
  if (ws_bytes < apply_bytes(*grid, nvec)) {
    set_error("workspace too small: need " + std::to_string(apply_bytes(*grid, nvec)) + " bytes");
    return HKP_E_WORKSPACE;
  }
  HKP_TRY(check_device());
  FilterArgs a{};
  a.grid = *grid;
  a.mat = *mat;
  a.V = V_eV;
  a.strain = strain;
  for (int i = 0; i < 3; ++i) a.B[i] = B_T[i];
  a.nvec = nvec;
  a.X = X;
  a.Y_old = Y_old;
  a.Y = Y;
  a.alpha = alpha;
  a.shift = shift;
  a.beta = beta;
  a.precision = precision;
  a.workspace = workspace;
  a.stream = hip_stream;
  a.st = autotuned(*grid, nvec, precision == HKP_PREC_MIXED,
                   stencil_variant(strain != nullptr, B_T));
  return guarded([&]() { return run_filter_step(a); });
}

size_t hkp_filter_step2_workspace_bytes(const hkp_grid* grid, int32_t nvec) {
  if (check_grid(grid) != HKP_OK) return 0;
  if (nvec < 1) {
    set_error("nvec >= 1 required");
    return 0;
  }
  return apply2_bytes(*grid, nvec);
}

int hkp_filter_step2(const hkp_grid* grid, const hkp_material* mat, const double* V_eV,
                     const double* strain, const double B_T[3], int32_t nvec, const void* X,
                     const void* Y_old, void* Y1, void* Y2, const double alpha[2],
                     const double shift[2], const double beta[2], void* workspace,
                     size_t ws_bytes, void* hip_stream, int32_t* passes) {
  HKP_TRY(check_grid(grid));
  HKP_TRY(check_material(mat));
  HKP_TRY(check_field(B_T));
  if (nvec < 1 || !V_eV || !X || !Y1 || !Y2 || !workspace || !alpha || !shift || !beta) {
    set_error("nvec >= 1 and non-NULL V, X, Y1, Y2, alpha, shift, beta, workspace required");
    return HKP_E_ARG;
  }
  for (int i = 0; i < 2; ++i)
    if (!std::isfinite(alpha[i]) || !std::isfinite(shift[i]) || !std::isfinite(beta[i])) {
      set_error("alpha, shift, beta must be finite");
      return HKP_E_ARG;
    }
  if (beta[0] != 0.0 && !Y_old) {
    set_error("beta[0] != 0 needs Y_old");
    return HKP_E_ARG;
  }
  if (Y1 == Y2 || Y1 == X || Y2 == X || (Y_old && (Y1 == Y_old || Y2 == Y_old))) {
    set_error("Y1 and Y2 must be distinct from each other and from X and Y_old");
    return HKP_E_ARG;
  }
  if (ws_bytes < apply2_bytes(*grid, nvec)) {
    set_error("workspace too small: need " + std::to_string(apply2_bytes(*grid, nvec)) +
              " bytes");
    return HKP_E_WORKSPACE;
  }
  HKP_TRY(check_device());
  Filter2Args a{};
  a.grid = *grid;
  a.mat = *mat;
  a.V = V_eV;
  a.strain = strain;
  for (int i = 0; i < 3; ++i) a.B[i] = B_T[i];
  a.nvec = nvec;
  a.X = X;
  a.Y_old = Y_old;
  a.Y1 = Y1;
  a.Y2 = Y2;
  for (int i = 0; i < 2; ++i) {
    a.alpha[i] = alpha[i];
    a.shift[i] = shift[i];
    a.beta[i] = beta[i];
  }
  a.workspace = workspace;
  a.stream = hip_stream;
  a.st = autotuned(*grid, nvec, true, stencil_variant(strain != nullptr, B_T));
  int np = 0;
  const int rc = guarded([&]() { return run_filter_step2(a, &np); });
  if (passes) *passes = np;
  return rc;
}

int hkp_apply(const hkp_grid* grid, const hkp_material* mat, const double* V_eV,
              const double* strain, const double B_T[3], int32_t nvec, const void* X, void* Y,
              int32_t precision, void* workspace, size_t ws_bytes, void* hip_stream) {
  return hkp_filter_step(grid, mat, V_eV, strain, B_T, nvec, X, nullptr, Y, 1.0, 0.0, 0.0,
                         precision, workspace, ws_bytes, hip_stream);
}

int hkp_gate_potential(int64_t N, int32_t G, const double* V_bg, const double* L,
                       const double* Vg, double* V_out, void* hip_stream) {
  if (N < 1 || G < 0 || !V_bg || !V_out || (G > 0 && (!L || !Vg))) {
    set_error("hkp_gate_potential: invalid arguments");
    return HKP_E_ARG;
  }
  HKP_TRY(check_device());
  return guarded([&]() {
    hipError_t e = launch_gate_potential(N, G, V_bg, L, Vg, V_out, (hipStream_t)hip_stream);
    if (e != hipSuccess) {
      set_error(hipGetErrorString(e));
      return HKP_E_HIP;
    }
    return HKP_OK;
  });
}

int hkp_hf_grad_noalloc(int64_t N, int32_t nev, const void* psi, const double* w, int32_t G,
                        const double* L, double* grad, void* hip_stream) {
  if (N < 1 || nev < 1 || !psi || !w || !L || !grad) {
    set_error("hkp_hf_grad_noalloc: invalid arguments (N >= 1, nev >= 1, non-NULL pointers)");
    return HKP_E_ARG;
  }
  if (G < 1 || (size_t)G * hf_partial_bytes(1) > hf_scratch_bytes()) {
    set_error("hkp_hf_grad_noalloc: G = " + std::to_string(G) + " outside 1..16 (the static "
              "scratch holds " + std::to_string(hf_scratch_bytes()) + " bytes of partial sums)");
    return HKP_E_ARG;
  }
  HKP_TRY(check_device());
  return guarded([&]() {
    double* partial = nullptr;
    hipError_t e = hf_scratch(&partial);
    if (e == hipSuccess)
      e = launch_hf_grad(N, nev, psi, w, G, L, partial, grad, (hipStream_t)hip_stream);
    if (e != hipSuccess) {
      set_error(hipGetErrorString(e));
      return HKP_E_HIP;
    }
    return HKP_OK;
  });
}

size_t hkp_hf_grad_workspace_bytes(int32_t G) {
  if (G < 1 || G > 16) {
    set_error("hkp_hf_grad: 1 <= G <= 16");
    return 0;
  }
  return hf_partial_bytes(G);
}

int hkp_hf_grad(int64_t N, int32_t nev, const void* psi, const double* w, int32_t G,
                const double* L, double* grad, void* workspace, size_t ws_bytes,
                void* hip_stream) {
  if (N < 1 || nev < 1 || G < 1 || G > 16 || !psi || !w || !L || !grad || !workspace) {
    set_error("hkp_hf_grad: invalid arguments (1 <= G <= 16)");
    return HKP_E_ARG;
  }
  if (ws_bytes < hf_partial_bytes(G)) {
    set_error("workspace too small: need " + std::to_string(hf_partial_bytes(G)) + " bytes");
    return HKP_E_WORKSPACE;
  }
  HKP_TRY(check_device());
  return guarded([&]() {
    hipError_t e = launch_hf_grad(N, nev, psi, w, G, L, (double*)workspace, grad,
                                  (hipStream_t)hip_stream);
    if (e != hipSuccess) {
      set_error(hipGetErrorString(e));
      return HKP_E_HIP;
    }
    return HKP_OK;
  });
}

int hkp_autotune(const hkp_grid* grid, int32_t nb, int32_t precision, int32_t with_strain,
                 int32_t with_field, void* workspace, size_t ws_bytes, void* hip_stream,
                 hkp_tune* out) {
  HKP_TRY(check_grid(grid));
  if (nb < 1 || nb > HKP_NB_MAX || !workspace || !out || with_field < 0 || with_field > 2 ||
      (precision != HKP_PREC_FP64 && precision != HKP_PREC_MIXED)) {
    set_error("hkp_autotune: invalid arguments");
    return HKP_E_ARG;
  }
  HKP_TRY(check_device());
  return guarded([&]() {
    return run_autotune(*grid, nb, precision == HKP_PREC_MIXED, with_strain != 0,
                        with_field, workspace, ws_bytes, hip_stream, out);
  });
}

int hkp_tuned_shape(const hkp_grid* grid, int32_t nb, int32_t precision, int32_t with_strain,
                    int32_t with_field, hkp_tune* out) {
  HKP_TRY(check_grid(grid));
  if (nb < 1 || nb > HKP_NB_MAX || !out || with_field < 0 || with_field > 2 ||
      (precision != HKP_PREC_FP64 && precision != HKP_PREC_MIXED)) {
    set_error("hkp_tuned_shape: invalid arguments");
    return HKP_E_ARG;
  }
  const double B[3] = {with_field ? 0.5 : 0.0, 0.0, with_field == 2 ? 0.5 : 0.0};
  const StencilTune t = autotuned(*grid, nb, precision == HKP_PREC_MIXED,
                                  stencil_variant(with_strain != 0, B));
  std::memset(out, 0, sizeof(*out));
  out->tile_y = t.tile_y;
  out->vgroup = t.vgroup;
  out->dma = t.dma;
  out->two_step_tx = t.t2x;
  out->two_step_ty = t.t2y;
  return HKP_OK;
}

int hkp_tune_cache_save(const char* path) {
  return guarded([&]() { return tune_cache_save(path); });
}

int hkp_tune_cache_load(const char* path) {
  return guarded([&]() { return tune_cache_load(path); });
}

void hkp_tune_cache_clear(void) { tune_cache_clear(); }

int hkp_autotune_block(const hkp_grid* grid, const hkp_material* mat, const hkp_opts* opts,
                       const double* V_eV, const double* strain, const double B_T[3],
                       const int32_t* candidates, int32_t ncand, void* workspace,
                       size_t ws_bytes, void* hip_stream, int32_t* nb_out,
                       double* seconds_out) {
  HKP_TRY(check_grid(grid));
  HKP_TRY(check_opts(grid, opts));
  if (!mat || !V_eV || !B_T || !candidates || !workspace || !nb_out || ncand < 1 ||
      ncand > 16) {
    set_error("hkp_autotune_block: invalid arguments (1 <= ncand <= 16, pointers non-NULL)");
    return HKP_E_ARG;
  }
  HKP_TRY(check_material(mat));
  HKP_TRY(check_field(B_T));
  const long long n6 = 6LL * grid->nx * grid->ny * grid->nz;
  int cmax = 0;
  for (int k = 0; k < ncand; ++k) {
    if (candidates[k] <= opts->nev || candidates[k] > HKP_NB_MAX || candidates[k] > n6) {
      set_error("hkp_autotune_block: every candidate must satisfy nev < nb <= min(64, 6 N)");
      return HKP_E_ARG;
    }
    cmax = std::max(cmax, (int)candidates[k]);
  }
  {
    hkp_opts o = *opts;
    o.nb = cmax;
    const size_t need = plan_bytes(make_plan(*grid, o, 1));
    if (ws_bytes < need) {
      set_error("workspace too small: need " + std::to_string(need) + " bytes");
      return HKP_E_WORKSPACE;
    }
  }
  HKP_TRY(check_device());
  return guarded([&]() {
    return run_autotune_block(*grid, *mat, *opts, V_eV, strain, B_T, candidates, ncand,
                              workspace, ws_bytes, hip_stream, nb_out, seconds_out);
  });
}

const char* hkp_last_error(void) { return g_err.c_str(); }

size_t hkp_soi_workspace_bytes(const hkp_grid* grid, int32_t M) {
  if (check_grid(grid) != HKP_OK) return 0;
  if (M < 1 || 3 * M > HKP_NB_MAX) {
    set_error("hkp_soi_matrix: 1 <= M <= 21");
    return 0;
  }
  const long long N = (long long)grid->nx * grid->ny * grid->nz;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  return al((size_t)3 * M * N * 16) + al(gram_partial_bytes(3 * M, N, 1)) +
         al((size_t)9 * M * M * 16);
}

int hkp_soi_matrix(const hkp_grid* grid, int32_t M, const void* phi, const double* E_eV,
                   double delta_so_eV, void* out, void* workspace, size_t ws_bytes,
                   void* hip_stream) {
  HKP_TRY(check_grid(grid));
  if (M < 1 || 3 * M > HKP_NB_MAX || !phi || !out || !workspace || !std::isfinite(delta_so_eV)) {
    set_error("hkp_soi_matrix: 1 <= M <= 21, finite delta_so, non-NULL phi, out, workspace");
    return HKP_E_ARG;
  }
  const size_t need = hkp_soi_workspace_bytes(grid, M);
  if (ws_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return HKP_E_WORKSPACE;
  }
  HKP_TRY(check_device());
  return guarded([&]() {
    const long long N = (long long)grid->nx * grid->ny * grid->nz;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    char* w = static_cast<char*>(workspace);
    double* comp = reinterpret_cast<double*>(w);
    double* partial = reinterpret_cast<double*>(w + al((size_t)3 * M * N * 16));
    double* O = reinterpret_cast<double*>(w + al((size_t)3 * M * N * 16) +
                                          al(gram_partial_bytes(3 * M, N, 1)));
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = launch_gather_components(N, M, phi, comp, s);
    const BlockDesc A{comp, N, 3 * M, 3LL * M * N};
    if (e == hipSuccess) e = launch_gram(A, A, 1, 1, partial, O, nullptr, s);
    if (e == hipSuccess) e = launch_soi_assemble(M, O, E_eV, delta_so_eV, out, s);
    if (e != hipSuccess) {
      set_error(hipGetErrorString(e));
      return HKP_E_HIP;
    }
    return HKP_OK;
  });
}

size_t hkp_ci_workspace_bytes(const hkp_grid* grid, int32_t M, const hkp_pgrid* pgrid) {
  if (check_grid(grid) != HKP_OK || check_pgrid(pgrid, grid) != HKP_OK) return 0;
  if (M < 1 || M > 5) {
    set_error("hkp_ci_solve: 1 <= M <= 5");
    return 0;
  }
  return ci_bytes(*grid, M, *pgrid);
}

int hkp_ci_solve(const hkp_grid* grid, int32_t M, const void* phi, const double* E_eV,
                 double delta_so_eV, const hkp_pgrid* pgrid, const double* eps_r,
                 const uint8_t* dirichlet, double cg_tol, int32_t cg_max_iter, double* eig_eV,
                 void* vecs, void* H_ci, void* coulomb, double* J_eV, void* workspace,
                 size_t ws_bytes, void* hip_stream, hkp_ci_stats* stats) {
  HKP_TRY(check_grid(grid));
  HKP_TRY(check_pgrid(pgrid, grid));
  if (M < 1 || M > 5 || !phi || !E_eV || !eps_r || !dirichlet || !eig_eV || !workspace ||
      !std::isfinite(delta_so_eV) || !finite_pos(cg_tol) || cg_max_iter < 1) {
    set_error("hkp_ci_solve: 1 <= M <= 5, non-NULL phi, E, eps_r, dirichlet, eig, workspace, "
              "finite delta_so, cg_tol > 0, cg_max_iter >= 1");
    return HKP_E_ARG;
  }
  const size_t need = ci_bytes(*grid, M, *pgrid);
  if (ws_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return HKP_E_WORKSPACE;
  }
  HKP_TRY(check_device());
  CIArgs a{};
  a.grid = *grid;
  a.M = M;
  a.phi = phi;
  a.E = E_eV;
  a.delta_so = delta_so_eV;
  a.pg = *pgrid;
  a.eps = eps_r;
  a.dir = dirichlet;
  a.cg_tol = cg_tol;
  a.cg_max_iter = cg_max_iter;
  a.eig = eig_eV;
  a.vecs = vecs;
  a.H = H_ci;
  a.coulomb = coulomb;
  a.J = J_eV;
  a.workspace = workspace;
  a.stream = hip_stream;
  return guarded([&]() { return run_ci(a, stats); });
}

size_t hkp_poisson_workspace_bytes(const hkp_pgrid* pgrid) {
  if (check_pgrid(pgrid, nullptr) != HKP_OK) return 0;
  return poisson_bytes(*pgrid);
}

int hkp_poisson(const hkp_pgrid* pgrid, double h_nm, const double* eps_r,
                const uint8_t* dirichlet, const double* phi_fixed, const double* rho,
                double* phi, double cg_tol, int32_t cg_max_iter, void* workspace,
                size_t ws_bytes, void* hip_stream, int32_t* cg_iters, double* cg_relres) {
  HKP_TRY(check_pgrid(pgrid, nullptr));
  if (!finite_pos(h_nm) || !finite_pos(cg_tol) || cg_max_iter < 1) {
    set_error("hkp_poisson: h > 0, cg_tol > 0, cg_max_iter >= 1");
    return HKP_E_ARG;
  }
  if (!eps_r || !dirichlet || !phi_fixed || !phi || !workspace) {
    set_error("hkp_poisson: eps_r, dirichlet, phi_fixed, phi and workspace must not be NULL");
    return HKP_E_ARG;
  }
  if (ws_bytes < poisson_bytes(*pgrid)) {
    set_error("workspace too small: need " + std::to_string(poisson_bytes(*pgrid)) + " bytes");
    return HKP_E_WORKSPACE;
  }
  HKP_TRY(check_device());
  PoissonArgs a{};
  a.pg = *pgrid;
  a.h = h_nm;
  a.eps = eps_r;
  a.dir = dirichlet;
  a.phi_fixed = phi_fixed;
  a.rho = rho;
  a.phi = phi;
  a.tol = cg_tol;
  a.max_iter = cg_max_iter;
  a.workspace = workspace;
  a.stream = hip_stream;
  int it = 0;
  double rr = 0.0;
  const int rc = guarded([&]() { return run_poisson(a, &it, &rr); });
  if (cg_iters) *cg_iters = it;
  if (cg_relres) *cg_relres = rr;
  return rc;
}

int hkp_occupancy(int32_t nev, const double* E_eV, double n_holes, double T_K, double* f,
                  double* mu_eV, void* hip_stream) {
  if (nev < 1 || nev > 64 || !E_eV || !f || !(n_holes >= 0.0 && n_holes <= nev) ||
      !finite_pos(T_K)) {
    set_error("hkp_occupancy: 1 <= nev <= 64, 0 <= n_holes <= nev, T > 0, non-NULL E and f");
    return HKP_E_ARG;
  }
  HKP_TRY(check_device());
  return guarded([&]() {
    hipError_t e = launch_occupancy(nev, E_eV, n_holes, kBoltzmann * T_K, f, mu_eV,
                                    (hipStream_t)hip_stream);
    if (e != hipSuccess) {
      set_error(hipGetErrorString(e));
      return HKP_E_HIP;
    }
    return HKP_OK;
  });
}

int hkp_hole_density(const hkp_grid* grid, int32_t nev, const void* psi, const double* f,
                     double* density, void* hip_stream) {
  HKP_TRY(check_grid(grid));
  if (nev < 1 || !psi || !f || !density) {
    set_error("hkp_hole_density: nev >= 1 and non-NULL psi, f, density");
    return HKP_E_ARG;
  }
  HKP_TRY(check_device());
  return guarded([&]() {
    const PGeom g{grid->nx, grid->ny, grid->nz, (long long)grid->nx * grid->ny * grid->nz};
    const double h = grid->h_nm;
    hipError_t e = launch_rho(g, 0, 0, 0, grid->nx, grid->ny, grid->nz, nev, psi, 6 * g.NP, f,
                              1.0 / (h * h * h), nullptr, nullptr, density,
                              (hipStream_t)hip_stream);
    if (e != hipSuccess) {
      set_error(hipGetErrorString(e));
      return HKP_E_HIP;
    }
    return HKP_OK;
  });
}

namespace {
// the loop's density is formed from six-component spinors: the spin-free
// orbital problem (three components per vector) is not a loop option
int check_sp_flags(const hkp_opts* o) {
  if (o->flags & HKP_FLAG_SPIN_FREE) {
    set_error("hkp_sp_solve: HKP_FLAG_SPIN_FREE is not supported in the self-consistent loop");
    return HKP_E_ARG;
  }
  return HKP_OK;
}
}  // namespace

size_t hkp_sp_workspace_bytes(const hkp_grid* grid, const hkp_opts* opts,
                              const hkp_pgrid* pgrid, const hkp_sp_opts* sp) {
  if (check_grid(grid) != HKP_OK || check_opts(grid, opts) != HKP_OK ||
      check_pgrid(pgrid, grid) != HKP_OK || check_sp_opts(sp, opts->nev) != HKP_OK ||
      check_sp_flags(opts) != HKP_OK)
    return 0;
  return sp_bytes(*grid, *opts, *pgrid, *sp);
}

int hkp_sp_solve(const hkp_grid* grid, const hkp_material* mat, const hkp_opts* opts,
                 const hkp_pgrid* pgrid, const hkp_sp_opts* sp, const double* V_off_eV,
                 const double* strain, const double B_T[3], const double* eps_r,
                 const uint8_t* dirichlet, const double* phi_fixed, const double* rho_fixed,
                 double* phi, double* eig_eV, void* psi, double* resid_eV, double* density,
                 void* workspace, size_t ws_bytes, void* hip_stream, hkp_sp_stats* stats) {
  HKP_TRY(check_grid(grid));
  HKP_TRY(check_material(mat));
  HKP_TRY(check_field(B_T));
  HKP_TRY(check_opts(grid, opts));
  HKP_TRY(check_pgrid(pgrid, grid));
  HKP_TRY(check_sp_opts(sp, opts->nev));
  HKP_TRY(check_sp_flags(opts));
  if (!V_off_eV || !eps_r || !dirichlet || !phi_fixed || !phi || !eig_eV || !workspace) {
    set_error("hkp_sp_solve: V_off, eps_r, dirichlet, phi_fixed, phi, eig and workspace "
              "must not be NULL");
    return HKP_E_ARG;
  }
  if ((opts->flags & HKP_FLAG_GRAPH) && hip_stream == nullptr) {
    set_error("HKP_FLAG_GRAPH needs a non-default stream (the legacy stream cannot be captured)");
    return HKP_E_ARG;
  }
  const size_t need = sp_bytes(*grid, *opts, *pgrid, *sp);
  if (ws_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return HKP_E_WORKSPACE;
  }
  HKP_TRY(check_device());
  SPArgs a{};
  a.grid = *grid;
  a.mat = *mat;
  a.opts = *opts;
  a.pg = *pgrid;
  a.sp = *sp;
  a.V_off = V_off_eV;
  a.strain = strain;
  for (int i = 0; i < 3; ++i) a.B[i] = B_T[i];
  a.eps = eps_r;
  a.dir = dirichlet;
  a.phi_fixed = phi_fixed;
  a.rho_fixed = rho_fixed;
  a.phi = phi;
  a.eig = eig_eV;
  a.psi = psi;
  a.resid = resid_eV;
  a.density = density;
  a.workspace = workspace;
  a.stream = hip_stream;
  return guarded([&]() { return run_sp(a, stats); });
}

size_t hkp_gmatrix_workspace_bytes(const hkp_grid* grid) {
  if (check_grid(grid) != HKP_OK) return 0;
  return gmatrix_bytes(*grid);
}

int hkp_gmatrix(const hkp_grid* grid, const hkp_material* mat, const double* V_eV,
                const double* strain, const void* psi, void* out, void* workspace,
                size_t ws_bytes, void* hip_stream) {
  HKP_TRY(check_grid(grid));
  HKP_TRY(check_material(mat));
  if (!V_eV || !psi || !out || !workspace) {
    set_error("hkp_gmatrix: non-NULL V, psi, out, workspace required");
    return HKP_E_ARG;
  }
  const size_t need = gmatrix_bytes(*grid);
  if (ws_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return HKP_E_WORKSPACE;
  }
  HKP_TRY(check_device());
  GMatrixArgs a{};
  a.grid = *grid;
  a.mat = *mat;
  a.V = V_eV;
  a.strain = strain;
  a.psi = psi;
  a.out = out;
  a.workspace = workspace;
  a.stream = hip_stream;
  {
    const double B0[3] = {0.0, 0.0, 0.0};
    a.st = autotuned(*grid, 16, false, stencil_variant(strain != nullptr, B0));
  }
  return guarded([&]() { return run_gmatrix(a); });
}

int hkp_st_model(const void* gm, const double* J_eV, const hkp_st_opts* opts, int32_t nB,
                 const double* B_T, void* points, void* H, void* hip_stream) {
  if (!gm || !J_eV || !opts || !B_T || !points || nB < 1 || nB > (1 << 24)) {
    set_error("hkp_st_model: 1 <= nB <= 2^24 and non-NULL gm, J, opts, B, points required");
    return HKP_E_ARG;
  }
  const double* n = opts->n_so;
  const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  if (!(nn > 0.0) || !std::isfinite(nn) || !(opts->lambda_so_nm > 0.0) ||
      !std::isfinite(opts->lambda_so_nm) || !std::isfinite(opts->d_nm)) {
    set_error("hkp_st_model: nonzero finite n_so, finite lambda_so > 0 and finite d required");
    return HKP_E_ARG;
  }
  HKP_TRY(check_device());
  return guarded([&]() {
    const double u[3] = {n[0] / nn, n[1] / nn, n[2] / nn};
    const hipError_t e = launch_st_model(gm, J_eV, u, opts->lambda_so_nm, opts->d_nm, nB, B_T,
                                         points, H, (hipStream_t)hip_stream);
    if (e != hipSuccess) {
      set_error(hipGetErrorString(e));
      return HKP_E_HIP;
    }
    return HKP_OK;
  });
}

void hkp_set_iter_callback(hkp_iter_fn fn, void* user) { set_iter_callback(fn, user); }

int hkp_poisson_preconditioner(int32_t kind) {
  if (kind != HKP_PRECOND_MULTIGRID && kind != HKP_PRECOND_JACOBI) {
    set_error("hkp_poisson_preconditioner: HKP_PRECOND_MULTIGRID or HKP_PRECOND_JACOBI");
    return HKP_E_ARG;
  }
  return set_poisson_precond(kind);
}

int hkp_version(void) { return 113; }

}  // extern "C"
