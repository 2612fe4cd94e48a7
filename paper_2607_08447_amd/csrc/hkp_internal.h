// Internal declarations shared by the host orchestration and the HIP kernels.
//
// Internal data layout (device, HBM):
//   spinor block   complex [vec][c][z][y][x], c = 0..5 in the |L S> basis
//                  |X up>,|Y up>,|Z up>,|X dn>,|Y dn>,|Z dn> (spin-major),
//                  x fastest; one (vec, c) slice is a contiguous 3-D field.
//   onsite fields  real [6][z][y][x]: d00 d11 d22 d12 d02 d01 of the orbital
//                  3x3 block V + H_eps (strain present), or [z][y][x] = V.
//   gauge          A' = (By (z-z0), Bz (x-x0) - Bx (z-z0), 0): links along z
//                  carry no phase, x-links a phase per plane, y-links a phase
//                  per (plane, column).  Related to the symmetric gauge of the
//                  ABI by psi_sym = exp(-i (e/hbar) chi) psi' with
//                  chi = -Bz XY/2 - By XZ/2 + Bx YZ/2 (coordinates about r0).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "hkp.h"

namespace hkp {

void set_error(const std::string& msg);   // thread-local message for hkp_last_error

// The hardware places workgroup wg on XCD wg % 8; this gives every XCD a
// contiguous run of logical workgroups (neighbouring data then shares an L2).
__device__ __forceinline__ int xcd_remap(int wg, int nwg) {
  const int x = wg & 7, idx = wg >> 3;
  const int per = nwg >> 3, rem = nwg & 7;
  return x * per + (x < rem ? x : rem) + idx;
}

// unit constants from CODATA 2018 (h, e exact; m0 = 9.1093837015e-31 kg),
// ten significant digits
constexpr double kE0 = 0.03809982116;         // hbar^2/(2 m0), eV nm^2
constexpr double kMuB = 5.788381806e-5;       // e hbar/(2 m0), eV/T
constexpr double kEoverHbar = 1.519267448e-3; // e/hbar, 1/(T nm^2)

// ---------------------------------------------------------------------------
// stencil constants (host-computed in double, converted to the kernel type)
// ---------------------------------------------------------------------------
template <typename T>
struct StencilConsts {
  T cLM, cM, czZ, cN8;   // face and edge coefficients
  T dgU, dgD;            // spin-diagonal onsite constant (kinetic centre + SO/Zeeman)
  T aUx, aUy, aUz;       // i (aU x v) term of the up block
  T aDx, aDy, aDz;       // i (aD x v) term of the down block
  T d3;                  // Delta/3 (spin-flip spin-orbit)
  T bx, by;              // mu_B Bx, mu_B By (spin-flip Zeeman)
};

StencilConsts<double> make_consts(const hkp_material& m, double h, const double B[3]);
template <typename T>
StencilConsts<T> cast_consts(const StencilConsts<double>& c);

// Chebyshev step coefficients, device array [batch][kmax][4] = alpha, shift, beta, pad
struct StepCoef {
  const double* coef;  // may be null: use the host values below
  int stride;          // doubles between batch members
  double alpha, shift, beta;
};

struct StencilLaunch {
  int nx, ny, nz;
  int nvec;              // vectors per Hamiltonian in this launch
  int batch;             // Hamiltonians
  const void* in;        // kernel-type complex block
  long long in_bstride;  // complex elements between Hamiltonians
  const void* old;       // may be null (beta = 0)
  int old_fp64;          // element type of old
  long long old_bstride;
  void* out;
  int out_fp64;
  long long out_bstride;
  const void* D;         // onsite fields (kernel type)
  long long D_bstride;   // reals between Hamiltonians
  int strain;            // D holds 6 arrays
  const void* wtab;      // [nz] complex, kernel type, or null (B = 0)
  const void* vtab;      // [nz][nx] complex
  int phase_general;     // Bz != 0: y-link phases vary along x
  StepCoef coef;
  const int* active;     // [batch] 0 = skip, or null
  const int* lock;       // [batch] vectors below this index are skipped, or null
  const int* work;       // [batch + 1] prefix sums of the vectors to process per member
                         // (vector lock[b] + i of member b is virtual vector work[b] + i);
                         // the grid covers nvec * batch vectors and only the first
                         // work[batch] are live, spread evenly over the XCDs. Or null.
  int tile_y;            // 1, 2, 4
  int vgroup;            // vectors of one tile side by side (1 vector-major, nvec tile-major)
  int dma;               // 1: rows staged global -> LDS directly (needs nx % 64 == 0)
  int zsplit;            // z ranges per (vector, tile): 0 never, 1 for small launches, 2 always
  int fp64;              // kernel type
  int ncomp = 6;         // components per vector: 6 (spinor) or 3 (spin-free orbital, no field)
};

hipError_t launch_stencil(const StencilLaunch& a, const StencilConsts<double>& c,
                          hipStream_t s);

// Two Chebyshev steps in one pass (FP32): Y1 = alpha1 (H - shift1) Y0 + beta1 Y_old,
// Y2 = alpha2 (H - shift2) Y1 + beta2 Y0, coefficients per member from the device
// table.  Y1 and Y2 must be distinct from Y0 and Y_old.
struct Stencil2Launch {
  int nx, ny, nz;
  int nvec, batch;
  const void* in;        // Y0, complex float
  const void* old;       // Y_old
  void* out1;            // Y1
  void* out2;            // Y2
  long long bstride;     // complex elements between Hamiltonians (all four blocks)
  const void* D;         // on-site fields, float
  long long D_bstride;
  int strain;
  const void* zero;      // >= 16 bytes of zeros in device memory
  const void* wtab;      // float phase tables, or null (B = 0)
  const void* vtab;
  int phase_general;     // Bz != 0: not supported by this kernel
  const double* coef1;   // [batch][...]: alpha, shift, beta of the first step, or null
  const double* coef2;   // of the second (both null: host1 / host2 below)
  int coef_stride;
  double host1[3], host2[3];
  const int* active;
  const int* lock;
  const int* work;
  int tile_x, tile_y;    // 16 x 12, 16 x 8 or 32 x 8; nx % tile_x == 0
  int vgroup;
};
bool stencil2_supported(const Stencil2Launch& a);
hipError_t launch_stencil2(const Stencil2Launch& a, const StencilConsts<double>& c,
                           hipStream_t s);

// ---------------------------------------------------------------------------
// field setup and boundary transforms
// ---------------------------------------------------------------------------
hipError_t launch_onsite(const hkp_material& m, int nx, int ny, int nz, int batch,
                         const double* V, long long V_bstride, const double* strain,
                         double* D64, float* D32, long long D_bstride, hipStream_t s);
hipError_t launch_phase_tables(int nx, int nz, double h, const double B[3], double* w64,
                               double* v64, float* w32, float* v32, hipStream_t s);
// ABI (J basis, symmetric gauge, [v][x][y][z][6]) <-> internal (LS, GPU gauge)
hipError_t launch_abi_to_internal(int nx, int ny, int nz, double h, const double B[3],
                                  int nvec, const void* abi, void* internal, int to_fp32,
                                  hipStream_t s);
hipError_t launch_internal_to_abi(int nx, int ny, int nz, double h, const double B[3],
                                  int nvec, int batch, const void* internal,
                                  long long in_bstride, void* abi, long long abi_bstride,
                                  hipStream_t s);
hipError_t launch_gate_potential(long long N, int G, const double* Vbg, const double* L,
                                 const double* Vg, double* out, hipStream_t s);
size_t hf_partial_bytes(int G);
// device address of this device's static partial-sum array (hf_blocks() x 16
// doubles), looked up once per device; never allocates
hipError_t hf_scratch(double** out);
size_t hf_scratch_bytes();
hipError_t launch_hf_grad(long long N, int nev, const void* psi, const double* w, int G,
                          const double* L, double* partial, double* grad, hipStream_t s);

// ---------------------------------------------------------------------------
// block linear algebra
// ---------------------------------------------------------------------------
struct BlockDesc {   // complex double block set: [batch][nvec][n]
  double* ptr;       // as doubles (re, im interleaved)
  long long n;       // complex elements per vector
  int nvec;
  long long bstride; // complex elements between Hamiltonians
};

// partial Gram of A^H B over chunks (MFMA f64); out: [batch][nb_a][nb_b] complex
int gram_chunks(long long n, int batch);
size_t gram_partial_bytes(int nb, long long n, int batch);
hipError_t launch_gram(const BlockDesc& A, const BlockDesc& B, int hermitian, int batch,
                       double* partial, double* out, const int* active, hipStream_t s);
// X[:, 0:nout] <- X[:, 0:nin] Q (Q complex [batch][nin][nout], column-major by
// output), in place allowed
hipError_t launch_rotate(const BlockDesc& X, const BlockDesc& Y, int nin, int nout,
                         const double* Q, int batch, const int* active, hipStream_t s);
// workgroups per member of a rotation (and partial sums per vector of launch_ritz)
int rotate_blocks(long long n, int batch);
// Rayleigh-Ritz rotation with Ritz vectors Q of X^H W (W = H X): X <- X Q in
// place, r2[b][j] = || (W Q)_j - theta_j (X Q)_j ||^2 and the first filter step
// Y1 = alpha (W Q - shift X Q) (coefficients from theta, the upper bound and,
// for the product form, its first root),
// FP32 into out32 where f32[b], else FP64 in place into W; W Q is not stored.
// partial holds batch x nb x rotate_blocks(n, batch) doubles
hipError_t launch_ritz(const BlockDesc& X, const BlockDesc& W, int nb, const double* Q,
                       const double* theta, const double* bounds, const double* roots,
                       const int* f32, float* out32, int batch, double* partial, double* r2,
                       const int* active, hipStream_t s);
hipError_t launch_cast(const void* in, int in_fp64, void* out, int out_fp64, long long count,
                       hipStream_t s);
hipError_t launch_random_block(double* X, long long n, int nvec, int batch, long long bstride,
                               unsigned long long seed, hipStream_t s);
// per-vector complex dot products (conj(a) . b) and norms for Lanczos
hipError_t launch_dots(const double* a, const double* b, long long n, int batch,
                       long long bstride, double* partial, double* out, hipStream_t s);
hipError_t launch_lanczos_update(double* w, const double* v, const double* vprev, long long n,
                                 int batch, long long bstride, const double* alpha,
                                 const double* beta, hipStream_t s);
hipError_t launch_scale(double* v, long long n, int batch, long long bstride,
                        const double* norm2, hipStream_t s);

// ---------------------------------------------------------------------------
// small dense eigenproblems (one workgroup per matrix)
// ---------------------------------------------------------------------------
// mode 0 (RR):   A Hermitian nb x nb -> eigenvalues theta (ascending) and
//                eigenvectors Q (columns), written over A's buffer layout
// mode 1 (SVQB): A = Gram S -> T = D U diag(lambda)^-1/2, D = diag(S)^-1/2
// SVQB mode: again[b] (if given) is set to 1 when the Gram matrix is so ill
// conditioned that a second pass is needed (and the member is active)
// C = op(A) B per member (op: A if adj = 0, A^H if adj = 1), nb x nb complex
// row-major; herm: store the Hermitian part; C must not alias A or B
// the product form's roots (Leja order, on [-1, 1]) into the device table
constexpr int kMaxDegree = 200;
struct RootTable {
  double x[kMaxDegree];
};
hipError_t launch_set_roots(double* dst, const RootTable& t, int m, hipStream_t s);
hipError_t launch_small_gemm(const double* A, int adj, const double* B, double* C, int nb,
                             int batch, long long mat_stride, int herm, const int* active,
                             hipStream_t s);
hipError_t launch_set_identity(double* C, int nb, int batch, long long mat_stride,
                               const int* active, hipStream_t s);
hipError_t launch_heev(double* A, int nb, int batch, long long mat_stride, double* evals,
                       double* out, int mode, int* status, const int* active, hipStream_t s,
                       int* again = nullptr);

// first step of the scaled Chebyshev filter: damp [a_cut, b_up], value 1 at the
// lowest Ritz value a0; Y1 = alpha (H - shift) X (the later steps' coefficients
// follow from the same e, c and sigma_1)
// (acut: the largest Ritz value, kept at least 1e-9 of the interval above a0)
__device__ __forceinline__ void cheb_interval(double bup, double a0, double& acut, double* e,
                                              double* c, double* sigma1) {
  if (acut - a0 < 1e-9 * (bup - a0)) acut = a0 + 1e-9 * (bup - a0);
  *e = 0.5 * (bup - acut);
  *c = 0.5 * (bup + acut);
  *sigma1 = *e / (a0 - *c);
}
// first step Y1 = alpha (H - shift) X: of the recurrence, or (roots != null) the
// first factor of the product form, (H - r_0) / (a0 - r_0) with r_0 the first
// root mapped onto [a_cut, b_up]
__device__ __forceinline__ void cheb_first_coef(double bup, double a0, double acut,
                                                const double* roots, double* alpha,
                                                double* shift) {
  double e, c, s1;
  cheb_interval(bup, a0, acut, &e, &c, &s1);
  if (roots) {
    const double r = c + e * roots[0];
    *alpha = 1.0 / (a0 - r);
    *shift = r;
  } else {
    *alpha = s1 / e;
    *shift = c;
  }
}

// control: convergence flags, next Chebyshev coefficients
struct Control {
  double* theta;     // [batch][nb]
  double* r2;        // [batch][nb] squared residuals
  double* coef;      // [batch][kmax*4]
  double* bounds;    // [batch][4]: b_upper, a_cut, a0, last rmax
  int* flags;        // [batch][8]: done, fp64, stagnation, iters, nconv, switch iter, lock
  int* active;       // [batch] not converged
  int* act32;        // [batch] not converged, FP32 filter
  int* act64;        // [batch] not converged, FP64 filter
  int* lock;         // [batch] leading vectors left out of the filter (converged pairs)
  int* sw;           // [batch] next filter FP64 but its first step was written in FP32
                     // (the member left the FP32 filter at this control step)
  const double* roots;   // product form: the next filter's m Chebyshev roots on [-1, 1]
                         // in Leja order (null: three-term recurrence)
  int* work;         // [3][batch + 1] prefix sums of vectors to process per member:
                     // FP32 filter, FP64 filter (both after the lock), whole block
};
// rebuild Control::work from the active masks and lock counts
hipError_t launch_worktable(const Control& c, int batch, int nb, hipStream_t s);
hipError_t launch_control(const Control& c, int batch, int nb, int nev, int degree,
                          int kmax, double tol, int mixed, int allow_switch, int allow_lock,
                          int iter, hipStream_t s);
hipError_t launch_finish(const double* theta, const double* r2, int nb, int nev, int batch,
                         double* eig, double* resid, hipStream_t s);
hipError_t launch_check_finite(const double* x, long long count, int* flag, hipStream_t s);
hipError_t launch_fill_int(int* p, int count, int value, hipStream_t s);

// ---------------------------------------------------------------------------
// spin-free basis (orbital vectors [v][x][y][z][3] complex) and spin-orbit matrix
// ---------------------------------------------------------------------------
hipError_t launch_orbital_to_internal(int nx, int ny, int nz, int nvec, const void* orb,
                                      double* internal, hipStream_t s);
hipError_t launch_internal_to_orbital(int nx, int ny, int nz, int nvec, int batch,
                                      const double* internal, long long in_bstride, void* orb,
                                      long long out_bstride, hipStream_t s);
// [M][N][3] -> [3M][N] (component b of orbital i is vector 3 i + b)
hipError_t launch_gather_components(long long N, int M, const void* orb, double* comp,
                                    hipStream_t s);
// O: [3M][3M] complex overlaps; out: [2M][2M] complex, index 2 i + s; E may be null
hipError_t launch_soi_assemble(int M, const double* O, const double* E, double delta_so,
                               void* out, hipStream_t s);

// ---------------------------------------------------------------------------
// self-consistent loop: Poisson (conjugate gradients), occupancy, density,
// Anderson mixing.  Poisson-box arrays are real [px][py][pz] (z fastest).
// ---------------------------------------------------------------------------
constexpr int kRedBlocks = 16384;  // workgroups of the grid-stride kernels (max)
constexpr double kEoverEps0 = 1.602176634e-19 / 8.8541878128e-12 * 1e9;   // V nm
constexpr double kBoltzmann = 8.617333262e-5;                             // eV/K

struct PGeom {
  int px, py, pz;
  long long NP;
};

// conjugate-gradient scalars, device resident (no host round trip per step)
struct CGState {
  double rz, rr, bb, thr, alpha, beta;
  int it, done, breakdown, pad;
};

// multigrid preconditioner of the Poisson CG (2 x 2 x 2 aggregation, Galerkin
// coarse operators; see sp.hip): levels down to at most kMGCoarsest nodes
constexpr int kMGMaxLevels = 12;
constexpr int kMGCoarsest = 256;
constexpr double kMGOmega = 0.9;       // damped-Jacobi weight (D^-1 A has spectrum in [0, 2])
constexpr double kMGAlpha = 1.8;       // finest-level scaling of the coarse correction
constexpr int kMGCoarseSweeps = 30;    // even
// the coarse tail of the V-cycle: up to kMGTailLevels levels of at most
// kMGTailNodes nodes each (the last is the coarsest), solved by one workgroup
constexpr int kMGTailLevels = 3;
constexpr int kMGTailNodes = 1024;
struct MGLevel {
  int nx, ny, nz;
  long long N;
  long long off;    // offset of the level in the coefficient arrays
  long long voff;   // offset of the level in a system's coarse vectors (levels >= 1)
};
struct MGPlan {
  int nlev;
  MGLevel lv[kMGMaxLevels];
  long long total;    // coefficient entries over all levels
  long long vtotal;   // coarse-vector entries of one system (levels >= 1)
  int tail;           // first level of the tail (1 <= tail <= nlev - 1)
};
struct MGData {
  MGPlan plan;
  double *ax, *ay, *az, *diag, *dinv;   // [plan.total]
  double *b, *u;                        // [nrhs][plan.vtotal]
  double* partial_rz;                   // [nrhs][kRedBlocks]
};
MGPlan mg_plan(const PGeom& g);
// level 0 from the CG's link coefficients, then every coarser level
hipError_t launch_mg_setup(const PGeom& g, const double* cx, const double* cy, const double* cz,
                           const uint8_t* dir, const MGData& m, hipStream_t s);
// after launch_cg_init: z and the starting r.z from the V-cycle
hipError_t launch_mg_start(const PGeom& g, const MGData& m, const double* r, double* z,
                           CGState* st, int nrhs, hipStream_t s);

int sp_blocks(long long n);
size_t sp_partial_doubles(int nrhs = 1);   // partial-sum scratch of the SP launchers
// link coefficients cx, cy, cz (+x, +y, +z links), D^-1 (0 on electrodes) and
// the number of electrode nodes (*n_dir, device)
hipError_t launch_pcoef(const PGeom& g, double h, const double* eps, const uint8_t* dir,
                        double* cx, double* cy, double* cz, double* dinv, double* partial,
                        double* n_dir, hipStream_t s);
// phi (in: guess) gets its electrode values (phi_fixed null: grounded); r = b - L phi,
// z = D^-1 r, p = 0, and the CG state (stop when |r| <= tol |b|).  nrhs systems at
// once: rho, phi, r, z, p (and p_new, q below) hold nrhs vectors NP apart, st nrhs
// states, partial sp_partial_doubles(nrhs)
hipError_t launch_cg_init(const PGeom& g, const double* cx, const double* cy, const double* cz,
                          const double* dinv, const uint8_t* dir, const double* phi_fixed,
                          const double* rho, double scale, double* phi, double* r, double* z,
                          double* p, double* partial, double tol, CGState* st, hipStream_t s,
                          int nrhs = 1);
// one CG iteration (no-op once st->done): p_new = z + beta p_old, q = L p_new,
// phi += alpha p_new, r -= alpha q, z = D^-1 r (Jacobi, in place) or z = V-cycle(r)
// (multigrid: the new r is written to z's buffer and the new z to r's, so the
// next iteration takes the two buffers the other way round)
hipError_t launch_cg_iter(const PGeom& g, const double* cx, const double* cy, const double* cz,
                          const double* dinv, const uint8_t* dir, double* z,
                          const double* p_old, double* p_new, double* q, double* phi,
                          double* r, double* partial, int max_iter, CGState* st,
                          hipStream_t s, int nrhs = 1, const struct MGData* mg = nullptr);
hipError_t launch_occupancy(int nev, const double* E, double n_holes, double kT, double* f,
                            double* mu, hipStream_t s);
// rho (P grid, may be null) = rho_fixed (may be null) + hole density embedded at
// (ox, oy, oz); density (S grid, nm^-3, may be null).  psi: ABI layout
// [nev][nx][ny][nz][6] complex with vstride complex entries between vectors.
hipError_t launch_rho(const PGeom& g, int ox, int oy, int oz, int nx, int ny, int nz, int nev,
                      const void* psi, long long vstride, const double* f, double inv_h3,
                      const double* rho_fixed, double* rho, double* density, hipStream_t s);
hipError_t launch_extract(int nx, int ny, int nz, const PGeom& g, int ox, int oy, int oz,
                          const double* V_off, const double* phi, double* V, hipStream_t s);
// configuration interaction: right-hand sides [2P][NP] of the P = M(M+1)/2 pair
// densities (real, imaginary parts), the pair potentials at the Schroedinger grid
// as complex [P][NS], pair products [M*M][NS], the determinant matrix [K][K] and
// the full tensor (ik|jl) [M][M][M][M] (complex)
hipError_t launch_pair_rhs(const PGeom& g, int ox, int oy, int oz, int nx, int ny, int nz, int M,
                           const void* phi, double h, double* rhs, hipStream_t s);
hipError_t launch_pair_potential_gather(const PGeom& g, int ox, int oy, int oz, int nx, int ny,
                                        int nz, int P, const double* V, double* Vc,
                                        hipStream_t s);
hipError_t launch_pair_product(long long NS, int M, const void* phi, double* A, hipStream_t s);
hipError_t launch_ci_assemble(int M, const double* hsp, const double* Cs, double* H,
                              hipStream_t s);
hipError_t launch_coulomb_expand(int M, const double* Cs, double* C, hipStream_t s);
hipError_t launch_exchange(const double* E, double* J, hipStream_t s);
// F = phi_out - phi_in, *delta = max |F| (device)
hipError_t launch_residual_max(const PGeom& g, const double* phi_in, const double* phi_out,
                               double* F, double* partial, double* delta, hipStream_t s);
// Anderson step over k stored entries (slots 0..k-1) of an m-slot history; the
// current (x, F) is stored at `slot`; m = 0: linear mixing
hipError_t launch_anderson(const PGeom& g, int k, int m, int slot, double mixing, double* x,
                           const double* F, double* histX, double* histF, double* G,
                           double* dots, double* gamma, double* partial, hipStream_t s);

// g-matrices: an internal block of 44 spinors (LS, B = 0) whose slots 0-3 hold the
// four states; slots 4 (a + 1) + v <- r_a psi_v (r about the box centre),
// slots 32 + 4 b + v <- Z_b psi_v (Zeeman matrix per tesla); the post kernel turns
// the 16 x 44 Gram product of slots 0-15 against 0-43 (slots 16-31 = H_0 of 0-15)
// into an hkp_gmatrix_result
hipError_t launch_position_weight(int nx, int ny, int nz, double h, double* buf, hipStream_t s);
hipError_t launch_zeeman_derivative(long long N, double kappa, double* buf, hipStream_t s);
hipError_t launch_gmatrix_post(const double* G, void* out, hipStream_t s);
hipError_t launch_st_model(const void* gm, const double* J, const double n_so[3], double lambda,
                           double d, int nB, const double* B, void* pts, void* H, hipStream_t s);

}  // namespace hkp
