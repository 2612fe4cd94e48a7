// Host-side solver interface used by the C ABI layer.
#pragma once

#include <functional>
#include <stdexcept>

#include "hkp_internal.h"

namespace hkp {

// a failed HIP call inside the host orchestration (mapped to HKP_E_HIP)
struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

// launch shape of the stencil kernel: rows per tile, vectors of one tile run
// side by side (1: vector-major order), rows staged global -> LDS directly
struct StencilTune {
  int tile_y = 4;
  int vgroup = 1;
  int dma = 0;
  int zsplit = 1;   // 0 never, 1 when a launch has few live workgroups, 2 always
  // FP32 filter: tile of the two-step kernel (two recurrence steps per pass),
  // 0 = one step per pass
  int t2x = 0, t2y = 0;
};

// the FP32 filter of this grid may run two steps per pass (spinor vectors,
// nx a multiple of the two-step kernel's tile width)
inline bool two_step_grid(int nx, int ncomp) { return ncomp == 6 && nx % 16 == 0; }

struct Plan {
  int nx, ny, nz;
  double h;
  long long N, n6;   // grid points, complex unknowns per vector (ncomp N)
  int ncomp;         // 6 (spinor) or 3 (spin-free orbital)
  int batch, nev, nb, degree;   // degree: fixed value or the ramp's maximum
  bool degree_fixed;
  bool mixed;
  bool two_step;   // FP32 filter in two-step passes (the workspace holds their outputs)
  bool product;    // filter in product form over the polynomial's roots (else recurrence)
  StencilTune st;
};

struct SolveArgs {
  Plan plan;
  hkp_material mat;
  const double* V;
  const double* strain;
  double B[3];
  const void* X0;
  double* eig;
  void* psi;
  double* resid;
  void* workspace;
  void* stream;
  double tol;
  int max_iter;
  int flags;
  unsigned long long seed;
  StencilTune st;
  int graph_chunk;  // iterations per recorded graph
  // > 0: an upper bound of the spectrum of H (one Hamiltonian), used instead of
  // the Lanczos estimate (the self-consistent loop carries it across iterations)
  double bound_hint = 0.0;
};

struct FilterArgs {
  hkp_grid grid;
  hkp_material mat;
  const double* V;
  const double* strain;
  double B[3];
  int nvec;
  const void* X;
  const void* Y_old;
  void* Y;
  double alpha, shift, beta;
  int precision;
  void* workspace;
  void* stream;
  StencilTune st;
};

int default_nb(int nev, long long n6);
// block size for opts->nb == 0: the autotuned one for this grid, nev and
// precision if hkp_autotune_block ran in this process, else default_nb
int block_size(const hkp_grid& g, const hkp_opts& o);
int run_autotune_block(const hkp_grid& g, const hkp_material& mat, const hkp_opts& o,
                       const double* V, const double* strain, const double B[3],
                       const int* cand, int ncand, void* ws, size_t ws_bytes, void* stream,
                       int* nb_out, double* seconds_out);
Plan make_plan(const hkp_grid& g, const hkp_opts& o, int batch);
size_t plan_bytes(const Plan& p);
int run_solve(const SolveArgs& a, hkp_stats* stats);
// the calling thread's progress callback of its eigensolves (NULL: none)
void set_iter_callback(hkp_iter_fn fn, void* user);
size_t apply_bytes(const hkp_grid& g, int nvec);
int run_filter_step(const FilterArgs& a);
// two recurrence steps in FP32 (one pass when the two-step kernel supports the
// grid and field, else two); *passes receives 1 or 2
struct Filter2Args {
  hkp_grid grid;
  hkp_material mat;
  const double* V;
  const double* strain;
  double B[3];
  int nvec;
  const void* X;
  const void* Y_old;
  void* Y1;
  void* Y2;
  double alpha[2], shift[2], beta[2];
  void* workspace;
  void* stream;
  StencilTune st;
};
size_t apply2_bytes(const hkp_grid& g, int nvec);
int run_filter_step2(const Filter2Args& A, int* passes);
int guarded(const std::function<int()>& f);
// stencil variant of a launch: strain on/off and the link-phase kind
int stencil_variant(bool strain, const double B[3]);
StencilTune autotuned(const hkp_grid& g, int nb, bool mixed, int variant);
// the FP32 filter of this grid and block size runs in two-step passes: the
// autotuner chose them for some variant (or HKP_STENCIL2 forces a tile)
bool two_step_tuned(const hkp_grid& g, int nb);
// the autotuners' caches in a text file (hkp_tune_cache_save / _load / _clear)
int tune_cache_save(const char* path);
int tune_cache_load(const char* path);
void tune_cache_clear();
int run_autotune(const hkp_grid& g, int nb, bool mixed, bool strain, int field, void* ws,
                 size_t ws_bytes, void* stream, hkp_tune* out);

// ---- self-consistent loop and its Poisson solve
struct PoissonArgs {
  hkp_pgrid pg;           // offsets unused
  double h;
  const double* eps;
  const uint8_t* dir;
  const double* phi_fixed;
  const double* rho;
  double* phi;            // in: guess, out: solution
  double tol;
  int max_iter;
  void* workspace;
  void* stream;
};
size_t poisson_bytes(const hkp_pgrid& pg);
int set_poisson_precond(int kind);   // returns the previous kind
int run_poisson(const PoissonArgs& a, int* iters, double* relres);

struct SPArgs {
  hkp_grid grid;
  hkp_material mat;
  hkp_opts opts;
  hkp_pgrid pg;
  hkp_sp_opts sp;
  const double* V_off;
  const double* strain;
  double B[3];
  const double* eps;
  const uint8_t* dir;
  const double* phi_fixed;
  const double* rho_fixed;
  double* phi;
  double* eig;
  void* psi;
  double* resid;
  double* density;
  void* workspace;
  void* stream;
};
size_t sp_bytes(const hkp_grid& g, const hkp_opts& o, const hkp_pgrid& pg,
                const hkp_sp_opts& sp);
int run_sp(const SPArgs& a, hkp_sp_stats* stats);

// ---- two-hole configuration interaction
struct CIArgs {
  hkp_grid grid;
  int M;
  const void* phi;
  const double* E;
  double delta_so;
  hkp_pgrid pg;
  const double* eps;
  const uint8_t* dir;
  double cg_tol;
  int cg_max_iter;
  double* eig;
  void* vecs;
  void* H;
  void* coulomb;
  double* J;
  void* workspace;
  void* stream;
};
size_t ci_bytes(const hkp_grid& g, int M, const hkp_pgrid& pg);
int run_ci(const CIArgs& a, hkp_ci_stats* stats);

// ---- g-matrices of the double dot's doublets
struct GMatrixArgs {
  hkp_grid grid;
  hkp_material mat;
  const double* V;
  const double* strain;
  const void* psi;
  void* out;
  void* workspace;
  void* stream;
  StencilTune st;
};
size_t gmatrix_bytes(const hkp_grid& g);
int run_gmatrix(const GMatrixArgs& a);

}  // namespace hkp
