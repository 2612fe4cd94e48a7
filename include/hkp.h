/*
 * hkp.h -- C ABI of an MI355X (gfx950) solver for the lowest hole eigenpairs
 * of the finite-difference 6x6 Luttinger-Kohn k.p Hamiltonian
 *
 *     H_NI = H_LK + H_PB + V_DQD            (paper, Sec. II.C, Eq. HNI)
 *
 * with Bir-Pikus strain, Zeeman and Peierls-phase magnetic terms and an
 * electrostatic potential, discretised on a homogeneous grid with Dirichlet
 * walls (Sec. II.B).  The eigenpairs are found by Chebyshev-filtered subspace
 * iteration with Rayleigh-Ritz (the Rayleigh-Chebyshev method named in
 * Sec. II.B).  This is the Schroedinger half of the paper's self-consistent
 * Schroedinger-Poisson loop (Fig. 2a).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  Units: energy eV, length nm, magnetic field T, gate voltage V.
 *  Hole picture: H = -H_valence, so bound hole states are the LOWEST
 *  eigenvalues.
 *  Grid: interior points r = ((i+1)h, (j+1)h, (k+1)h), 0 <= i < nx, ...;
 *  psi = 0 one spacing outside the grid (hard wall).  nx, ny, nz >= 1 and
 *  N = nx ny nz <= 2^31 / 6 (larger grids are rejected with HKP_E_ARG).
 *  Scalar fields (V, lever arms): double [nx][ny][nz], C order (z fastest).
 *  Strain: double [nx][ny][nz][6], symmetric tensor components in the order
 *  xx, yy, zz, yz, xz, xy (tensor, not engineering, shear).
 *  Spinor blocks (X0, psi, apply operands): complex double (re, im pairs)
 *  [nvec][nx][ny][nz][6]; the six components are |J, m_j> in the order
 *  |3/2,+3/2>, |3/2,+1/2>, |3/2,-1/2>, |3/2,-3/2>, |1/2,+1/2>, |1/2,-1/2>
 *  (the order listed in Sec. II.C).  Vector potential in the symmetric gauge
 *  A = B x (r - r0) / 2 about the box centre r0 = ((n+1)h/2, ...).
 *  Wavefunctions are normalised to sum over grid and components of |psi|^2 = 1.
 *
 *  Pointers documented "device" must be device (HBM) memory of the current
 *  HIP device; "host" pointers are read before the call returns.  The caller
 *  owns every buffer.  No entry point allocates device memory: scratch comes
 *  from the caller's workspace.  Work is enqueued on `hip_stream` (a
 *  hipStream_t, NULL = default stream); entry points that return results in
 *  host structs synchronise that stream before returning.
 *
 *  Return codes: 0 success, > 0 warning (results written), < 0 error (nothing
 *  valid written).  Inputs are validated before any GPU work is enqueued.
 *  hkp_last_error() returns a thread-local description of the last failure.
 */
#ifndef HKP_H
#define HKP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HKP_OK 0
#define HKP_W_NOT_CONVERGED 1   /* best Ritz pairs and their residuals written */
#define HKP_E_ARG (-1)          /* invalid argument (sizes, NULL, NaN/Inf input) */
#define HKP_E_WORKSPACE (-2)    /* workspace smaller than hkp_*_workspace_bytes */
#define HKP_E_NUMERICAL (-3)    /* breakdown of the orthonormalisation */
#define HKP_E_HIP (-4)          /* a HIP runtime call failed */
#define HKP_E_UNSUPPORTED (-5)  /* no GPU of the supported architecture */

#define HKP_NB_MAX 64           /* largest block size */

#define HKP_PREC_FP64 0         /* every step in double precision */
#define HKP_PREC_MIXED 1        /* FP32 filter; FP64 orthonormalisation, RR, residual */

#define HKP_FLAG_X0 1           /* use the caller's initial block X0 */
#define HKP_FLAG_GRAPH 2        /* record outer iterations once in a hipGraph and replay */
#define HKP_FLAG_NO_FP64_POLISH 4 /* mixed: never switch the filter to FP64 */
#define HKP_FLAG_NO_LOCK 8      /* filter every vector of the block, converged or not */
#define HKP_FLAG_X0_NEV 16      /* with HKP_FLAG_X0: X0 holds nev vectors per member (a
                                 * previous solve's psi); the block's other nb - nev
                                 * vectors are drawn at random from the seed */
#define HKP_FLAG_SPIN_FREE 64   /* the spin-free orbital problem H_0 = H_DKK + V + H'_PB
                                 * (Eq. H0, Sec. II.D): no spin-orbit term (delta_so is
                                 * taken as 0), B_T must be zero; each orbital level once;
                                 * X0 and psi are complex [n][nx][ny][nz][3] (X, Y, Z) */
#define HKP_FLAG_PSI_BLOCK 32   /* psi receives the whole final block of nb Ritz vectors
                                 * (ascending Ritz values; eig and resid still nev), the
                                 * initial block of a restart that keeps the guard vectors */
#define HKP_FLAG_CHEB_PRODUCT 128 /* evaluate the Chebyshev filter in product form over its
                                 * roots (Leja order; each step reads Y_k and writes
                                 * Y_k+1) instead of the scaled three-term recurrence
                                 * (each step reads Y_k and Y_k-1, writes Y_k+1): the
                                 * same polynomial (Sec. II.B) with a third fewer bytes
                                 * per step; its FP32 residual floor is about 2x the
                                 * recurrence's */

/* Grid: nx, ny, nz >= 1 points, spacing h (nm) > 0. */
typedef struct {
  int32_t nx, ny, nz;
  double h_nm;
} hkp_grid;

/* Material: Luttinger parameters, split-off energy Delta_0 (eV), isotropic
 * magnetic parameter kappa, deformation potentials a_v, b, d (eV)
 * (paper, Appendix A, Table I).  q (the cubic Zeeman term) is zero. */
typedef struct {
  double gamma1, gamma2, gamma3;
  double delta_so_eV;
  double kappa;
  double a_v_eV, b_eV, d_eV;
} hkp_material;

/* Solver options.  nb = 0 selects the autotuned block size; degree = 0 the
 * default degree schedule over the first outer iterations: 16, then 32, then
 * 96 in FP64, or in mixed precision 48 + nb bounded to [64, 96] (88 at nb 40). */
typedef struct {
  int32_t nev;        /* eigenpairs wanted, 1 <= nev < nb */
  int32_t nb;         /* subspace block size, nev < nb <= HKP_NB_MAX, nb <= 6 N */
  int32_t degree;     /* Chebyshev polynomial degree per outer iteration, 0 or 1..200
                         (an odd degree is raised to the next even one) */
  int32_t max_iter;   /* outer iterations before HKP_W_NOT_CONVERGED */
  double tol_eV;      /* convergence: ||H psi_n - E_n psi_n||_2 <= tol for n < nev */
  int32_t precision;  /* HKP_PREC_FP64 or HKP_PREC_MIXED */
  int32_t flags;      /* HKP_FLAG_* */
  uint64_t seed;      /* seed of the random initial block */
} hkp_opts;

typedef struct {
  int32_t iters;            /* outer iterations performed (max over a batch) */
  int32_t n_converged;      /* wanted states meeting tol (min over a batch) */
  int64_t n_hx_fp64;        /* column applications of H in FP64 (sum over a batch) */
  int64_t n_hx_fp32;        /* column applications of H in FP32 */
  int32_t fp64_switch_iter; /* mixed: first outer iteration filtered in FP64, -1 none */
  int32_t nb, degree;       /* values used (after autotuning) */
  double seconds;           /* wall time of the call */
  double t_setup, t_filter, t_orth, t_rr, t_resid; /* event-timed phases (eager mode); the
                                          residual norms are formed inside the Rayleigh-Ritz
                                          phase (t_rr), t_resid times the convergence control */
  double lambda_max_bound;  /* upper spectral bound used by the filter (eV) */
  /* stencil launches (filter steps and H X): algorithmic bytes moved -- the
   * spinor blocks read and written plus the on-site fields once per launch --
   * and, in eager mode with stats requested, their event-timed durations on
   * the solver's stream, split by arithmetic precision */
  double hx_bytes;                       /* all stencil launches */
  int64_t n_stencil32, n_stencil64;      /* timed launches */
  double t_stencil32, t_stencil64;       /* summed durations (s) */
  double bytes_stencil32, bytes_stencil64; /* algorithmic bytes of the timed launches */
  /* FP32 passes that perform two recurrence steps each (timed as above; bytes:
   * those of the two steps, each counted as a one-step launch counts them) */
  int64_t n_stencil32x2;
  double t_stencil32x2, bytes_stencil32x2;
  int32_t n_graph_launches; /* replays of the recorded iteration graph (HKP_FLAG_GRAPH) */
  int32_t n_host_syncs;     /* host waits on the solver's stream (flag read-backs,
                               the spectral bound, the input check, the final wait) */
} hkp_stats;

/* Autotuner result for the stencil (filter step) kernel on one shape. */
typedef struct {
  int32_t tile_y;      /* rows of the x-y tile (the tile is 64 x tile_y) */
  int32_t vgroup;      /* vectors of one tile run side by side (1: vector-major) */
  int32_t dma;         /* 1: halo-tile rows copied global -> LDS directly */
  int32_t two_step_tx; /* FP32: tile of the two-step pass (two recurrence steps per */
  int32_t two_step_ty; /* pass) if it beats two one-step passes, else 0 x 0 */
  int32_t reserved;
  double us_per_step;  /* measured time of one filter step over the block */
  double gbps;         /* algorithmic bytes / time */
  double us_per_step_two; /* per recurrence step with two-step passes (0: not chosen) */
} hkp_tune;

/* ---- Self-consistent Schroedinger-Poisson loop (Sec. II.B, Fig. 2a) ----
 *
 * Poisson box: px x py x pz points with the spacing h of the Schroedinger
 * grid, which occupies the points ox <= i < ox + nx (and likewise in y, z).
 * Box fields are double [px][py][pz], C order (z fastest).  The potential
 * phi (V) solves -div(eps_r grad phi) = (e/eps0) rho with rho in e/nm^3
 * (holes positive): 7-point finite differences, link permittivity the
 * harmonic mean of the two nodes' eps_r, electrode (Dirichlet) nodes held at
 * their given potential, no flux through any other outer face (Neumann).
 * The hole potential energy on the Schroedinger grid is V = V_off + phi (eV).
 * Each eigenstate holds at most one hole, with the Fermi-Dirac occupation
 * f_n = 1 / (1 + exp((E_n - mu) / kT)) and mu fixed by sum f_n = n_holes;
 * the hole density is p = sum_n f_n sum_c |psi_n,c|^2 / h^3 (nm^-3). */
typedef struct {
  int32_t px, py, pz;   /* Poisson box points, each >= 1, px py pz <= 2^31 */
  int32_t ox, oy, oz;   /* offset of the Schroedinger grid inside the box */
} hkp_pgrid;

#define HKP_SP_PHI0 1   /* start from the caller's phi (else the hole-free potential) */
#define HKP_SP_EXACT_EIG 2  /* every eigensolve to opts->tol (else: see hkp_sp_solve) */

typedef struct {
  double n_holes;        /* holes in the computed states, 0 <= n_holes <= nev */
  double temperature_K;  /* > 0 */
  double mixing;         /* Anderson damping a, 0 < a <= 1 */
  int32_t history;       /* Anderson history m, 0..8 (0: linear mixing) */
  int32_t max_iter;      /* loop iterations, >= 1 */
  double tol_V;          /* stop when max |phi_out - phi_in| <= tol_V (V), > 0 */
  double cg_tol;         /* Poisson CG: stop at |r| <= cg_tol |b|, > 0 */
  int32_t cg_max_iter;   /* CG iterations per Poisson solve, >= 1 */
  int32_t flags;         /* HKP_SP_* */
  double anneal_K;       /* 0 (off) or a temperature above temperature_K at which the
                            loop runs first; see hkp_sp_solve */
} hkp_sp_opts;

typedef struct {
  int32_t iters;              /* loop iterations (Schroedinger + Poisson passes) */
  int32_t converged;          /* 1 if max |phi_out - phi_in| <= tol_V */
  double delta_V;             /* last max |phi_out - phi_in| */
  double mu_eV;               /* Fermi level of the last iteration */
  double f_last;              /* occupation of the highest computed state (nev too
                                 small for the filling if it is not ~0) */
  int64_t cg_iters;           /* conjugate-gradient iterations, all Poisson solves */
  int32_t schroedinger_iters; /* eigensolver outer iterations, all solves */
  int32_t solve_status;       /* worst eigensolver status (HKP_OK or a warning) */
  int32_t poisson_status;     /* worst Poisson status (HKP_OK or a warning) */
  int32_t nb;                 /* eigensolver block size used */
  double seconds, t_schroedinger, t_poisson;   /* wall time: total, and by half */
  int32_t anneal_iters;       /* iterations at anneal_K (included in iters) */
} hkp_sp_stats;

/* Silicon parameters of Table I (Appendix A) with gamma3 = 1.446 in place of
 * the table's 1.21: gamma1 4.285, gamma2 0.339, Delta_0 0.044 eV, kappa -0.42,
 * a_v 2.46 eV, b -2.35 eV, d -5.32 eV. */
void hkp_default_material(hkp_material* m);
/* The unit constants the library computes with (host, no GPU work):
 * out[0] = hbar^2/(2 m0) in eV nm^2 (the kinetic scale of Eq. LK),
 * out[1] = mu_B in eV/T (Zeeman term), out[2] = e/hbar in 1/(T nm^2) (Peierls
 * phases); CODATA 2018 values to ten significant digits.  NULL is ignored. */
void hkp_unit_constants(double out[3]);
/* nev 8, nb 0, degree 0, max_iter 200, tol 1e-8 eV, FP64, flags 0, seed 1. */
void hkp_default_opts(hkp_opts* o);

/* Bytes of device workspace hkp_solve / hkp_solve_batch need for `batch`
 * Hamiltonians on `grid` with `opts` (nb = 0: the block size from
 * hkp_autotune_block if it ran for this grid, nev and precision, else
 * nev + max(8, nev/2) rounded up to 8).  Returns 0 on invalid arguments. */
size_t hkp_workspace_bytes(const hkp_grid* grid, const hkp_opts* opts, int32_t batch);

/* The block size a solve with these arguments uses (opts->nb, or with nb = 0
 * the autotuned or default value above): the leading extent of psi with
 * HKP_FLAG_PSI_BLOCK.  Returns 0 on invalid arguments. */
int32_t hkp_block_size(const hkp_grid* grid, const hkp_opts* opts);

/* Lowest opts->nev eigenpairs of H for one potential (paper Sec. II.B).
 * The block (opts->nb) must exceed nev by at least one degenerate cluster
 * above the wanted states (a Kramers pair at B = 0): the filter's lower cut
 * is the block's largest Ritz value, and a block that ends inside a
 * degenerate level cannot separate it (the solve then returns
 * HKP_W_NOT_CONVERGED with the best Ritz pairs found).
 *   V_eV      device double [nx][ny][nz]
 *   strain    device double [nx][ny][nz][6] or NULL (no strain)
 *   B_T       host double[3], magnetic field (T)
 *   X0        device complex double [nb][nx][ny][nz][6] used when
 *             opts->flags & HKP_FLAG_X0, else ignored (may be NULL);
 *             [nev][nx][ny][nz][6] with HKP_FLAG_X0_NEV as well (restart
 *             from a neighbouring solve's psi, as between the iterations
 *             of a Schroedinger-Poisson loop, Fig. 2a); its columns must be
 *             linearly independent: a starting block whose first
 *             orthonormalisation breaks down (repeated or dependent columns)
 *             gives HKP_E_NUMERICAL
 *   V_eV, strain: NaN or Inf anywhere gives HKP_E_ARG (checked on the device
 *             before the solve starts)
 *   eig_eV    device double [nev], ascending
 *   psi       device complex double [nev][nx][ny][nz][6] (may be NULL);
 *             [nb][nx][ny][nz][6] with HKP_FLAG_PSI_BLOCK
 *   resid_eV  device double [nev], ||H psi_n - E_n psi_n||_2 (may be NULL)
 *   workspace device, ws_bytes >= hkp_workspace_bytes(grid, opts, 1)
 *   stats     host, may be NULL
 * Returns HKP_OK, HKP_W_NOT_CONVERGED or an error. */
int hkp_solve(const hkp_grid* grid, const hkp_material* mat, const hkp_opts* opts,
              const double* V_eV, const double* strain, const double B_T[3],
              const void* X0, double* eig_eV, void* psi, double* resid_eV,
              void* workspace, size_t ws_bytes, void* hip_stream, hkp_stats* stats);

/* The same for `batch` Hamiltonians that differ only in the potential (a
 * gate-voltage sweep, Fig. 2f): V_eV is [batch][nx][ny][nz]; X0 (with
 * HKP_FLAG_X0) [batch][nb][nx][ny][nz][6], or [batch][nev][nx][ny][nz][6]
 * with HKP_FLAG_X0_NEV; eig_eV [batch][nev], psi
 * [batch][nev][nx][ny][nz][6] ([batch][nb]... with HKP_FLAG_PSI_BLOCK),
 * resid_eV [batch][nev]; batch <= 65535.
 * Every kernel of an outer iteration covers the whole batch in one launch;
 * with HKP_FLAG_GRAPH the iterations are recorded once as a hipGraph and
 * replayed, converged members turning into no-ops on the device. */
int hkp_solve_batch(const hkp_grid* grid, const hkp_material* mat, const hkp_opts* opts,
                    int32_t batch, const double* V_eV, const double* strain,
                    const double B_T[3], const void* X0, double* eig_eV, void* psi,
                    double* resid_eV, void* workspace, size_t ws_bytes, void* hip_stream,
                    hkp_stats* stats);

/* Progress of an eigensolve after an outer iteration (after each replayed chunk
 * of iterations with HKP_FLAG_GRAPH).  Arrays are host memory owned by the
 * library and valid during the call only; values are those of the last
 * Rayleigh-Ritz step (Sec. II.B), per batch member. */
typedef struct {
  int32_t iter;              /* outer iterations done */
  int32_t batch, nb, nev;
  const int32_t* nconv;      /* [batch] wanted states meeting tol */
  const int32_t* fp64;       /* [batch] 1 once the member's filter runs in FP64 */
  const double* ritz_eV;     /* [batch][nb] Ritz values, ascending */
  const double* resid_eV;    /* [batch][nb] residual norms ||H x - theta x|| */
} hkp_iter_info;
/* Returns nonzero to end the solve after this iteration (the results are then
 * written as after max_iter: HKP_W_NOT_CONVERGED unless every state converged). */
typedef int (*hkp_iter_fn)(const hkp_iter_info* info, void* user);

/* Registers fn (NULL: none) for the eigensolves that the calling host thread runs
 * from now on: hkp_solve, hkp_solve_batch and those inside hkp_sp_solve and
 * hkp_autotune_block.  Each call of fn costs one host wait on the solver's
 * stream and a copy of 2 nb doubles per member. */
void hkp_set_iter_callback(hkp_iter_fn fn, void* user);

/* Workspace of hkp_apply / hkp_filter_step for nvec vectors. */
size_t hkp_apply_workspace_bytes(const hkp_grid* grid, int32_t nvec);

/* Y = alpha (H - shift) X + beta Y_old  on nvec spinors: one step of the
 * Chebyshev filter of the Rayleigh-Chebyshev eigensolver (Sec. II.B), with H
 * the discretised H_NI of Eq. HNI (Sec. II.C: Luttinger-Kohn kinetic term,
 * Bir-Pikus strain, Zeeman and Peierls terms, potential V) on the grid of
 * Sec. II.B; alpha = 1, shift = beta = 0 gives Y = H X.
 *   X, Y      device complex double [nvec][nx][ny][nz][6], nvec >= 1
 *   Y_old     device, same layout, or NULL when beta == 0; may alias Y
 *   precision HKP_PREC_FP64 or HKP_PREC_MIXED (operands rounded to FP32 and
 *             the stencil evaluated in FP32; result returned in FP64) */
int hkp_filter_step(const hkp_grid* grid, const hkp_material* mat, const double* V_eV,
                    const double* strain, const double B_T[3], int32_t nvec,
                    const void* X, const void* Y_old, void* Y, double alpha, double shift,
                    double beta, int32_t precision, void* workspace, size_t ws_bytes,
                    void* hip_stream);

/* Two consecutive steps of the Chebyshev filter (Sec. II.B) in complex FP32
 * arithmetic, H as in hkp_filter_step:
 *     Y1 = alpha[0] (H - shift[0]) X  + beta[0] Y_old
 *     Y2 = alpha[1] (H - shift[1]) Y1 + beta[1] X
 * in one pass over the grid (temporal blocking: X and Y_old read once, Y1 and
 * Y2 written once) when the two-step kernel supports the grid and field (nx a
 * multiple of 16, B_T[2] == 0), else as two one-step passes.
 *   X, Y1, Y2 device complex double [nvec][nx][ny][nz][6]; Y_old the same or
 *             NULL when beta[0] == 0; Y1, Y2 distinct from each other and from
 *             X and Y_old (HKP_E_ARG otherwise).  Operands are rounded to FP32
 *             and the results returned in FP64.
 *   alpha, shift, beta  host double[2], finite
 *   workspace device, ws_bytes >= hkp_filter_step2_workspace_bytes(grid, nvec)
 *   passes    host, may be NULL: receives 1 (one two-step pass) or 2. */
size_t hkp_filter_step2_workspace_bytes(const hkp_grid* grid, int32_t nvec);
int hkp_filter_step2(const hkp_grid* grid, const hkp_material* mat, const double* V_eV,
                     const double* strain, const double B_T[3], int32_t nvec, const void* X,
                     const void* Y_old, void* Y1, void* Y2, const double alpha[2],
                     const double shift[2], const double beta[2], void* workspace,
                     size_t ws_bytes, void* hip_stream, int32_t* passes);

/* Y = H X with H the discretised Hamiltonian H_NI of Eq. HNI (Sec. II.C) on
 * the grid of Sec. II.B (hkp_filter_step with alpha 1, shift 0, beta 0). */
int hkp_apply(const hkp_grid* grid, const hkp_material* mat, const double* V_eV,
              const double* strain, const double B_T[3], int32_t nvec, const void* X,
              void* Y, int32_t precision, void* workspace, size_t ws_bytes,
              void* hip_stream);

/* V_out = V_bg + sum_g Vg[g] L[g]: a linear gate -> potential map producing the
 * V_DQD term of Eq. HNI (Sec. II.C) from gate voltages (lever-arm fields L_g).
 *   V_bg, V_out device double [N]; L device double [G][N]; Vg device double [G]. */
int hkp_gate_potential(int64_t N, int32_t G, const double* V_bg, const double* L,
                       const double* Vg, double* V_out, void* hip_stream);

/* Hellmann-Feynman gradient: grad[g] = sum_n w[n] sum_r sum_c |psi_{n,c}(r)|^2 L[g](r),
 * the derivative of sum_n w_n E_n with respect to the gate voltages.  V_DQD
 * enters Eq. HNI (Sec. II.C) as a diagonal term, and with the linear gate map
 * of hkp_gate_potential dH/dV_g = L_g(r) times the identity on the spinor
 * components, so dE_n/dV_g = <psi_n| L_g |psi_n>.
 *   psi  device complex double [nev][N][6]; w device double [nev];
 *   L    device double [G][N] (1 <= G <= 16); grad device double [G];
 *   workspace device, ws_bytes >= hkp_hf_grad_workspace_bytes(G) (block
 *   partial sums, reduced in a fixed order: the result is deterministic).
 * Exact for a degenerate pair only if both members carry equal weight. */
size_t hkp_hf_grad_workspace_bytes(int32_t G);
int hkp_hf_grad(int64_t N, int32_t nev, const void* psi, const double* w, int32_t G,
                const double* L, double* grad, void* workspace, size_t ws_bytes,
                void* hip_stream);

/* hkp_hf_grad without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, serving loops, harnesses that
 * forbid allocation).  The block partial sums go to a static device array of
 * 128 KiB (1024 x 16 doubles) that each GPU the library runs on holds until
 * the process ends; nothing is allocated or freed.  Every partial sum is
 * written before it is read, so nothing needs clearing between calls.  All
 * calls on one GPU share that array: calls that overlap in time on one GPU
 * (different streams or threads) race and must be serialised by the caller.
 * Same arguments, layouts and result as hkp_hf_grad; G outside 1..16 (more
 * partial sums than the array holds) is rejected with HKP_E_ARG. */
int hkp_hf_grad_noalloc(int64_t N, int32_t nev, const void* psi, const double* w, int32_t G,
                        const double* L, double* grad, void* hip_stream);

/* Time the filter-step kernel's launch shapes for this grid and block size,
 * cache the fastest and report it.  The stencil variant timed: strain on or
 * off (with_strain), and with_field 0 (B = 0), 1 (B along x: link phases
 * uniform over a z-plane) or 2 (B with a z component: the general phase
 * kernel).  The cache lives for the process, keyed by shape, nb, precision
 * and variant; a solve or filter step whose variant was not tuned uses the
 * shape tuned for another variant of the same shape, nb and precision.
 * Needs workspace >= hkp_workspace_bytes(grid, opts{nb}, 1). */
int hkp_autotune(const hkp_grid* grid, int32_t nb, int32_t precision, int32_t with_strain,
                 int32_t with_field, void* workspace, size_t ws_bytes, void* hip_stream,
                 hkp_tune* out);

/* Block size by measurement: one complete solve of this Hamiltonian (opts:
 * nev, tolerance, precision, degree, max_iter; nb and graph/X0 flags ignored)
 * for each of the ncand (1..16) candidate block sizes, each nev < nb <=
 * min(64, 6N), timed to convergence.  The fastest converged candidate is
 * written to *nb_out and cached for the process per (grid, nev, precision):
 * hkp_solve, hkp_solve_batch and hkp_workspace_bytes with opts->nb == 0 then
 * use it.  seconds_out (host, ncand, may be NULL) receives each candidate's
 * time (negated if it did not converge).  Needs workspace >=
 * hkp_workspace_bytes(grid, opts{nb = largest candidate}, 1).  Returns
 * HKP_OK, HKP_W_NOT_CONVERGED (no candidate converged; nothing cached) or an
 * error. */
int hkp_autotune_block(const hkp_grid* grid, const hkp_material* mat, const hkp_opts* opts,
                       const double* V_eV, const double* strain, const double B_T[3],
                       const int32_t* candidates, int32_t ncand, void* workspace,
                       size_t ws_bytes, void* hip_stream, int32_t* nb_out,
                       double* seconds_out);

/* The launch shape a solve or filter step on this grid and block size would
 * use (the autotuned one for this variant, else one tuned for another variant
 * of the same shape, nb and precision, else the default), without timing
 * anything; host only.  with_strain, with_field as in hkp_autotune; the us and
 * gbps fields of out are 0.  Returns HKP_OK or HKP_E_ARG. */
int hkp_tuned_shape(const hkp_grid* grid, int32_t nb, int32_t precision, int32_t with_strain,
                    int32_t with_field, hkp_tune* out);

/* The autotuners' choices across processes: hkp_tune_cache_save writes every
 * cached launch shape (hkp_autotune) and block size (hkp_autotune_block) to a
 * text file, keyed by grid, block size or nev, precision and stencil variant,
 * under the current device's architecture name; hkp_tune_cache_load reads such
 * a file and takes the entries written for the current device's architecture
 * (others are skipped: a choice timed on one device is not carried to
 * another).  Host only; the caller owns the path.  Both return the number of
 * entries written or taken (>= 0), or HKP_E_ARG (NULL path, file not
 * readable/writable, malformed line: nothing is taken from a malformed file).
 * hkp_tune_cache_clear empties both caches of this process. */
int hkp_tune_cache_save(const char* path);
int hkp_tune_cache_load(const char* path);
void hkp_tune_cache_clear(void);

/* Workspace of hkp_soi_matrix for M orbitals on `grid`. */
size_t hkp_soi_workspace_bytes(const hkp_grid* grid, int32_t M);

/* Spin-orbit matrix of M spin-free orbitals (Eq. H1, Fig. 2d-e): out[2i+s][2j+t] =
 * <phi_i s| H_SO |phi_j t> with H_SO = (delta_so / 3)(1 - sum_a sigma_a (x) L_a) on
 * every grid point, (L_a)_bc = -i eps_abc on (X, Y, Z), s = 0 up, 1 down; plus
 * E_i on the diagonal when E is given (the single-particle part of the
 * configuration-interaction Hamiltonian in the basis phi_i (x) s).
 *   phi   device complex double [M][nx][ny][nz][3] (hkp_solve with
 *         HKP_FLAG_SPIN_FREE), 1 <= M <= 21
 *   E_eV  device double [M] or NULL
 *   out   device complex double [2M][2M]
 * The component overlaps are reduced in a fixed order (deterministic). */
int hkp_soi_matrix(const hkp_grid* grid, int32_t M, const void* phi, const double* E_eV,
                   double delta_so_eV, void* out, void* workspace, size_t ws_bytes,
                   void* hip_stream);

/* ---- Two-hole configuration interaction (Sec. II.D, Eq. Phi, Fig. 2d-f) ----
 * Determinants |u v>, u < v (lexicographic), of the 2M spin-orbitals u = 2i + s
 * of M spin-free orbitals.  Pair densities rho_ik = sum_b conj(phi_i,b) phi_k,b / h^3
 * get their potentials V_ik from the Poisson problem of hkp_poisson with every
 * electrode grounded (all M(M+1)/2 pairs solved together, real and imaginary
 * parts as separate right-hand sides); (ik|jl) = sum_r h^3 rho_ik V_jl (eV);
 * <uv|wx> = delta(s_u, s_w) delta(s_v, s_x) (i_u i_w | i_v i_x); the matrix is
 * <uv|H|wx> = h_uw d_vx + h_vx d_uw - h_ux d_vw - h_vw d_ux + <uv|wx> - <uv|xw>
 * with h = diag(E) (x) 1 + the spin-orbit matrix (hkp_soi_matrix), and
 * J = mean(E_1, E_2, E_3) - E_0 of its ascending spectrum. */
typedef struct {
  int64_t cg_iters;        /* CG iterations of the batched pair-potential solve (max over systems) */
  double cg_relres;        /* largest final |r| / |b| */
  int32_t poisson_solves;  /* nonzero real right-hand sides solved together, M^2 (the
                              imaginary parts of the M self pairs vanish and stop at once) */
  int32_t determinants;    /* K = M (2M - 1) */
  double t_poisson, seconds;
} hkp_ci_stats;

/* Workspace of hkp_ci_solve. */
size_t hkp_ci_workspace_bytes(const hkp_grid* grid, int32_t M, const hkp_pgrid* pgrid);

/*   phi       device complex double [M][nx][ny][nz][3] orthonormal spin-free orbitals,
 *             1 <= M <= 5 (K <= 45)
 *   E_eV      device double [M] their energies
 *   pgrid, eps_r, dirichlet  the Poisson box as in hkp_poisson / hkp_sp_solve
 *   eig_eV    device double [K], ascending
 *   vecs, H_ci  device complex double [K][K] or NULL: eigenvectors (column k =
 *             eigenvector k, row-major) and the matrix itself
 *   coulomb   device complex double [M][M][M][M] (ik|jl), or NULL
 *   J_eV      device double [1] or NULL (written when K >= 4)
 * Returns HKP_OK, HKP_W_NOT_CONVERGED (a pair potential missed cg_tol) or an error. */
int hkp_ci_solve(const hkp_grid* grid, int32_t M, const void* phi, const double* E_eV,
                 double delta_so_eV, const hkp_pgrid* pgrid, const double* eps_r,
                 const uint8_t* dirichlet, double cg_tol, int32_t cg_max_iter, double* eig_eV,
                 void* vecs, void* H_ci, void* coulomb, double* J_eV, void* workspace,
                 size_t ws_bytes, void* hip_stream, hkp_ci_stats* stats);

/* ---- g-matrices of the double dot and the effective two-spin model
 * (Sec. III: Eqs. HB, J_QD, J_anis) ----
 * The g-matrix of a Kramers doublet {u1, u2}: to first order in B the
 * Hamiltonian restricted to the doublet is (mu_B / 2) sum_ab sigma_a g_ab B_b,
 * so g_ab = Re tr(sigma_a M_b) / mu_B with M_b = <u_i| dH/dB_b |u_j>.  dH/dB_b
 * is the derivative of the whole Hamiltonian (Zeeman and Peierls terms) at
 * B = 0, in the symmetric gauge about the doublet's own centre of charge.  The
 * dots' doublets are the eigenvectors of the position x within the span of the
 * bonding and antibonding doublets (lower x = left).  g depends on the basis of
 * its doublet through a rotation on the left only; the symmetric g-tensor
 * sgn(det g) (g^T g)^(1/2) and the singular values of g do not. */
typedef struct {
  double g[4][3][3];        /* bonding, antibonding, left, right: row a = Pauli, column b = field */
  double g_sym[4][3][3];    /* symmetric g-tensors */
  double centre_nm[4][3];   /* centres of charge, about the box centre */
  double kramers[4][3];     /* tr M_b / mu_B: zero for a Kramers doublet */
  double E_eV[4];           /* <psi_i|H|psi_i> of the four input states */
  double delta_eV;          /* antibonding minus bonding doublet energy */
  double t_eV;              /* tunnel coupling |Delta| / sqrt(2) */
  double d_nm;              /* distance between the left and right centres */
} hkp_gmatrix_result;

/* Workspace of hkp_gmatrix: 44 spinor blocks of the grid plus small buffers. */
size_t hkp_gmatrix_workspace_bytes(const hkp_grid* grid);

/*   psi   device complex double [4][nx][ny][nz][6] (|J m_j>, as hkp_solve returns at
 *         B = 0): the bonding doublet (states 0, 1) and the antibonding doublet
 *         (states 2, 3), orthonormal; V_eV, strain (may be NULL) and mat as in hkp_solve
 *   out   device hkp_gmatrix_result
 * Returns HKP_OK or an error; nothing is allocated. */
int hkp_gmatrix(const hkp_grid* grid, const hkp_material* mat, const double* V_eV,
                const double* strain, const void* psi, void* out, void* workspace,
                size_t ws_bytes, void* hip_stream);

/* Effective two-spin model of Eq. HB for nB fields, one thread each, from the
 * left and right symmetric g-tensors and t of an hkp_gmatrix_result:
 *   R(theta) = rotation by theta about n_so, theta_so = d / lambda_so;
 *   b_bar = mu_B (R(-theta_so) g_L + R(theta_so) g_R) B / 2, delta_b likewise with
 *   a minus sign, delta E_Z = |delta_b|; U - eps = 2 t^2 / J;
 *   the 5 x 5 matrix in the basis S(0,2), S(1,1), T+, T-, T0 and its spectrum;
 *   J_hat = J R(-2 theta_so); J~ = R_L J_hat R_R^T, R_L the rotation about
 *   n_L x z that takes n_L = g_L B / |g_L B| to z (the lab frame if g_L B = 0);
 *   |J_perp| = |(J~xx + J~yy, J~xy - J~yx)| / 2, J_par = J~zz. */
typedef struct {
  double n_so[3];           /* spin-orbit axis, any nonzero length */
  double lambda_so_nm;      /* spin-orbit length, > 0 */
  double d_nm;              /* inter-dot distance; <= 0: the result's d_nm */
} hkp_st_opts;

typedef struct {
  double bbar_eV[3], dbar_eV[3];   /* b_bar and delta_b */
  double dEz_eV;                   /* |delta_b| */
  double E_eV[5];                  /* spectrum of the 5 x 5 matrix, ascending */
  double Jtilde_eV[3][3];          /* exchange matrix in the qubit frames */
  double J_perp_eV, J_par_eV;
} hkp_st_point;

/*   gm    device hkp_gmatrix_result (from hkp_gmatrix)
 *   J_eV  device double [1], the exchange at the detuning of interest (nonzero;
 *         hkp_ci_solve writes one)
 *   B_T   device double [nB][3], 1 <= nB <= 2^24
 *   points device hkp_st_point [nB]; H device complex double [nB][5][5] or NULL */
int hkp_st_model(const void* gm, const double* J_eV, const hkp_st_opts* opts, int32_t nB,
                 const double* B_T, void* points, void* H, void* hip_stream);

/* Preconditioner of every Poisson conjugate-gradient solve that follows in this
 * process (hkp_poisson, hkp_sp_solve, hkp_ci_solve); the solution to the given
 * tolerance does not depend on it, the iteration count does.
 *   HKP_PRECOND_MULTIGRID (default): one V-cycle per iteration over 2 x 2 x 2
 *     aggregation levels with Galerkin coarse operators and damped-Jacobi smoothing
 *     (a symmetric positive-definite preconditioner).
 *   HKP_PRECOND_JACOBI: the diagonal.
 * Returns the previous choice, or HKP_E_ARG for an unknown kind.  Not to be
 * changed while another thread runs a Poisson solve. */
#define HKP_PRECOND_MULTIGRID 0
#define HKP_PRECOND_JACOBI 1
int hkp_poisson_preconditioner(int32_t kind);

/* Workspace of hkp_poisson for this box. */
size_t hkp_poisson_workspace_bytes(const hkp_pgrid* pgrid);

/* One Poisson solve on the box (offsets unused): preconditioned conjugate
 * gradients (hkp_poisson_preconditioner) from the guess in phi.
 *   eps_r, phi_fixed, rho  device double [px][py][pz] (rho may be NULL: 0)
 *   dirichlet  device uint8 [px][py][pz], 1 = electrode node; at least one
 *              (a box without one is reported as HKP_E_ARG after the
 *              coefficient pass, the only check that reads device data)
 *   phi        device double [px][py][pz]; in: finite guess, out: solution
 *              (electrode nodes set to phi_fixed)
 *   cg_iters, cg_relres  host, may be NULL: iterations and final |r|/|b|
 * On a stream other than the legacy default stream the iterations run as a
 * recorded hipGraph.  The library keeps the last recorded graph of each host
 * thread (until the process ends) and replays it while the next call on that
 * thread passes the same workspace, phi and dirichlet pointers, box, cg_max_iter,
 * preconditioner and device; the graph holds pointers, never values, so the
 * buffers' contents may change between calls.
 * Returns HKP_OK, HKP_W_NOT_CONVERGED (cg_max_iter reached) or an error. */
int hkp_poisson(const hkp_pgrid* pgrid, double h_nm, const double* eps_r,
                const uint8_t* dirichlet, const double* phi_fixed, const double* rho,
                double* phi, double cg_tol, int32_t cg_max_iter, void* workspace,
                size_t ws_bytes, void* hip_stream, int32_t* cg_iters, double* cg_relres);

/* Fermi-Dirac occupations of nev (1..64) hole levels E_eV (device) holding
 * n_holes (0..nev) at temperature T_K > 0: f (device [nev]) and mu_eV (device
 * double, may be NULL); mu by 200 bisection steps on sum f = n_holes. */
int hkp_occupancy(int32_t nev, const double* E_eV, double n_holes, double T_K, double* f,
                  double* mu_eV, void* hip_stream);

/* Hole density on the Schroedinger grid, density (device double [nx][ny][nz],
 * nm^-3) = sum_n f[n] sum_c |psi_n,c|^2 / h^3; psi device complex double
 * [nev][nx][ny][nz][6] (either basis), f device double [nev], nev >= 1. */
int hkp_hole_density(const hkp_grid* grid, int32_t nev, const void* psi, const double* f,
                     double* density, void* hip_stream);

/* Workspace of hkp_sp_solve. */
size_t hkp_sp_workspace_bytes(const hkp_grid* grid, const hkp_opts* opts,
                              const hkp_pgrid* pgrid, const hkp_sp_opts* sp);

/* The self-consistent loop (Fig. 2a): from phi_in (the hole-free potential,
 * or the caller's phi with HKP_SP_PHI0) each iteration solves for the lowest
 * opts->nev eigenpairs of H(V_off + phi_in) (hkp_solve with opts; from the
 * second iteration on restarted from the previous iteration's whole block),
 * occupies them, forms the hole density and solves Poisson for phi_out;
 * it stops when max |phi_out - phi_in| <= tol_V, otherwise the next phi_in
 * comes from Anderson mixing: phi_in + a F - (dX + a dF) g with F = phi_out -
 * phi_in, dX and dF the differences to the m previous inputs and residuals,
 * and g the least-squares minimiser of |F - dF g|.  Unless HKP_SP_EXACT_EIG is
 * set, an eigensolve stops at the residual max(opts->tol, min(1e-4 eV, 0.01 x
 * the previous max |phi_out - phi_in|)) (the first one at 1e-4 eV from the
 * hole-free start, at opts->tol from a caller's phi), and a Poisson solve at
 * max(cg_tol, min(1e-6, 0.01 x that change)); when the loop meets tol_V after
 * such looser solves it makes one more pass at the same potential with
 * opts->tol and cg_tol, so the returned results always meet both.
 * With sp->anneal_K > temperature_K the loop first runs at anneal_K until
 * max |phi_out - phi_in| <= max(tol_V, 1 mV), then goes on at temperature_K from
 * that potential (the eigensolves keep restarting from the last block; the
 * Anderson history starts afresh).  It converges to the same fixed point; a
 * higher temperature makes the occupations of nearly degenerate levels, and so
 * the map from potential to density, smooth, which keeps the mixing from
 * wandering between near-degenerate charge configurations (for two holes in a
 * double dot at 1.5 K, anneal_K = 15 K).  Iterations at both temperatures count
 * towards max_iter.
 *   V_off      device double [nx][ny][nz], band offset (e.g. the oxide step), eV
 *   strain, B_T as in hkp_solve
 *   eps_r, dirichlet, phi_fixed  as in hkp_poisson; rho_fixed device [px][py][pz]
 *              fixed charge (e/nm^3, e.g. ionised dopants) or NULL
 *   phi        device double [px][py][pz]; out: the last phi_in, the potential
 *              the returned eigenpairs belong to
 *   eig_eV, psi, resid_eV  as in hkp_solve (psi, resid may be NULL)
 *   density    device double [nx][ny][nz] hole density of the last iteration, or NULL
 *   stats      host, may be NULL
 * opts->flags: HKP_FLAG_GRAPH, HKP_FLAG_NO_FP64_POLISH, HKP_FLAG_NO_LOCK apply to
 * every eigensolve; X0 flags are ignored.  Returns HKP_OK, HKP_W_NOT_CONVERGED
 * (max_iter reached, or an eigensolve did not converge) or an error. */
int hkp_sp_solve(const hkp_grid* grid, const hkp_material* mat, const hkp_opts* opts,
                 const hkp_pgrid* pgrid, const hkp_sp_opts* sp, const double* V_off_eV,
                 const double* strain, const double B_T[3], const double* eps_r,
                 const uint8_t* dirichlet, const double* phi_fixed, const double* rho_fixed,
                 double* phi, double* eig_eV, void* psi, double* resid_eV, double* density,
                 void* workspace, size_t ws_bytes, void* hip_stream, hkp_sp_stats* stats);

/* Thread-local message of the last error (never NULL). */
const char* hkp_last_error(void);

/* ABI version (major * 100 + minor). */
int hkp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HKP_H */
