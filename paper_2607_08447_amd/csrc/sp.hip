// Kernels of the self-consistent Schroedinger-Poisson loop (paper Sec. II.B,
// Fig. 2a): the electrostatic potential from Poisson's equation by
// preconditioned conjugate gradients (a multigrid V-cycle, or the diagonal), the
// configuration interaction's pair potentials, Fermi-Dirac occupancy of the hole
// states, the hole density, and Anderson mixing of the potential.
//
// Poisson box layout (device, HBM): real [px][py][pz], x slowest and z fastest
// (the ABI layout, so nothing is transposed on the way in or out).  Link
// coefficients c = eps_link / h^2 are stored per node for its +x, +y and +z
// links (eps_link: harmonic mean of the two nodes' eps_r, zero for a link that
// would leave the box -- the field-free outer faces).  Electrode nodes keep
// their potential; every CG vector is zero on them.
//
// All of these kernels stream through memory once per call: they are HBM-bound
// and run one node per thread (grid-stride beyond kRedBlocks workgroups); the
// stencil-shaped ones give every XCD a contiguous range of nodes, so that the
// x- and y-neighbours a node reads are in the L2 its neighbours filled.
// Per-workgroup partial sums are reduced in a fixed order by one workgroup
// (the results do not depend on timing).
#include <hip/hip_runtime.h>

#include "hkp_internal.h"

namespace hkp {

namespace {

constexpr int kThreads = 256;

struct Geo {
  int px, py, pz;
  unsigned sx;    // py * pz (x stride; boxes hold < 2^31 nodes)
  unsigned sy;    // pz (y stride)
  double ipy, ipz;   // 1 / py, 1 / pz (host-computed)
};

__device__ __forceinline__ Geo geo(int px, int py, int pz, double ipy, double ipz) {
  return Geo{px, py, pz, (unsigned)py * (unsigned)pz, (unsigned)pz, ipy, ipz};
}

// n / d for n < 2^31 from a double reciprocal, corrected to the exact floor
// (the product is within a tiny fraction of n / d, so one step either way
// suffices); integer division by a runtime divisor costs far more
__device__ __forceinline__ unsigned udiv(unsigned n, unsigned d, double inv) {
  unsigned q = (unsigned)((double)n * inv);
  const unsigned long long qd = (unsigned long long)q * d;
  if (qd > n) --q;
  else if (qd + d <= n) ++q;
  return q;
}

// (x, y, z) of box node i
__device__ __forceinline__ void coords(unsigned i, const Geo& g, int& x, int& y, int& z) {
  const unsigned q = udiv(i, g.sy, g.ipz);   // x * py + y
  z = (int)(i - q * g.sy);
  x = (int)udiv(q, (unsigned)g.py, g.ipy);
  y = (int)(q - (unsigned)x * (unsigned)g.py);
}

__device__ __forceinline__ double harmonic(double a, double b) { return 2.0 * a * b / (a + b); }

constexpr int kRedThreads = 1024;   // the one workgroup that reduces partial sums

// block sum of NV values over NT threads; thread 0 writes them to out[0..NV)
template <int NV, int NT = kThreads>
__device__ __forceinline__ void block_sums(double (&v)[NV], double* out) {
  __shared__ double sh[NV][NT / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = v[k];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) sh[k][w] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int i = 0; i < NT / 64; ++i) s += sh[k][i];
      out[k] = s;
    }
  }
}

// sums of nblk partial rows (stride NV) by one workgroup of kRedThreads, fixed order
// (thread t adds rows t, t + kRedThreads, ... in turn).  Eight rows per thread are
// loaded before any is added (a clamped index and a zero stand in past the end),
// so a thread waits on memory once per eight rows rather than once per row.
template <int NV>
__device__ __forceinline__ void reduce_partials(const double* partial, int nblk, double* out) {
  constexpr int kBatch = 8;
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  for (int b0 = threadIdx.x; b0 < nblk; b0 += kBatch * kRedThreads) {
    double t[kBatch][NV];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int b = b0 + u * kRedThreads;
      const long long row = b < nblk ? b : nblk - 1;
#pragma unroll
      for (int k = 0; k < NV; ++k) t[u][k] = partial[row * NV + k];
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
#pragma unroll
      for (int k = 0; k < NV; ++k)
        if (b0 + u * kRedThreads < nblk) v[k] += t[u][k];
  }
  block_sums<NV, kRedThreads>(v, out);
}

// ---------------------------------------------------------------------------
// Poisson: link coefficients and the Jacobi preconditioner
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
pcoef_kernel(unsigned NP, int px, int py, int pz, double ipy, double ipz, double inv_h2,
             const double* __restrict__ eps, const uint8_t* __restrict__ dir, double* cx,
             double* cy, double* cz, double* dinv, double* partial) {
  const Geo g = geo(px, py, pz, ipy, ipz);
  double nd = 0.0;   // electrode nodes (checked on the host: at least one)
  for (unsigned i = xcd_remap(blockIdx.x, gridDim.x) * kThreads + threadIdx.x; i < NP;
       i += gridDim.x * kThreads) {
    int x, y, z;
    coords(i, g, x, y, z);
    const double e = eps[i];
    const double ax = x + 1 < px ? harmonic(e, eps[i + g.sx]) * inv_h2 : 0.0;
    const double ay = y + 1 < py ? harmonic(e, eps[i + g.sy]) * inv_h2 : 0.0;
    const double az = z + 1 < pz ? harmonic(e, eps[i + 1]) * inv_h2 : 0.0;
    const double bx = x > 0 ? harmonic(e, eps[i - g.sx]) * inv_h2 : 0.0;
    const double by = y > 0 ? harmonic(e, eps[i - g.sy]) * inv_h2 : 0.0;
    const double bz = z > 0 ? harmonic(e, eps[i - 1]) * inv_h2 : 0.0;
    cx[i] = ax;
    cy[i] = ay;
    cz[i] = az;
    const double diag = ax + ay + az + bx + by + bz;
    dinv[i] = (dir[i] || !(diag > 0.0)) ? 0.0 : 1.0 / diag;
    nd += dir[i] ? 1.0 : 0.0;
  }
  double v[1] = {nd};
  block_sums<1>(v, partial + blockIdx.x);
}

// sum over the in-box links of node i of c (u_i - u_j), with u_j from `val`
template <typename F>
__device__ __forceinline__ double link_sum(unsigned i, int x, int y, int z, const Geo& g,
                                           const double* __restrict__ cx,
                                           const double* __restrict__ cy,
                                           const double* __restrict__ cz, double ui, F val) {
  double s = 0.0;
  if (x + 1 < g.px) s += cx[i] * (ui - val(i + g.sx));
  if (x > 0) s += cx[i - g.sx] * (ui - val(i - g.sx));
  if (y + 1 < g.py) s += cy[i] * (ui - val(i + g.sy));
  if (y > 0) s += cy[i - g.sy] * (ui - val(i - g.sy));
  if (z + 1 < g.pz) s += cz[i] * (ui - val(i + 1));
  if (z > 0) s += cz[i - 1] * (ui - val(i - 1));
  return s;
}

// The six neighbours of node i at (x, y, z) in an nx x ny x nz box with strides
// sx, sy (order +x, -x, +y, -y, +z, -z), for branch-free stencils: indices clamped
// to i itself where the neighbour would lie outside the box, with that link's
// weight set to zero.  Every load of such a stencil is issued unconditionally, so
// a thread's loads go out back to back instead of one conditional round trip to
// memory per link.
struct Hood {
  unsigned j[6];
  bool in[6];
};
__device__ __forceinline__ Hood hood(unsigned i, int x, int y, int z, int nx, int ny, int nz,
                                     unsigned sx, unsigned sy) {
  Hood h;
  h.in[0] = x + 1 < nx;
  h.in[1] = x > 0;
  h.in[2] = y + 1 < ny;
  h.in[3] = y > 0;
  h.in[4] = z + 1 < nz;
  h.in[5] = z > 0;
  h.j[0] = h.in[0] ? i + sx : i;
  h.j[1] = h.in[1] ? i - sx : i;
  h.j[2] = h.in[2] ? i + sy : i;
  h.j[3] = h.in[3] ? i - sy : i;
  h.j[4] = h.in[4] ? i + 1 : i;
  h.j[5] = h.in[5] ? i - 1 : i;
  return h;
}
// weights of the six links from per-node +x, +y, +z link arrays (the link to the
// lower neighbour is stored there), zero outside the box
__device__ __forceinline__ void hood_weights(unsigned i, const Hood& h, const double* ax,
                                             const double* ay, const double* az,
                                             double (&c)[6]) {
  const double v[6] = {ax[i], ax[h.j[1]], ay[i], ay[h.j[3]], az[i], az[h.j[5]]};
#pragma unroll
  for (int q = 0; q < 6; ++q) c[q] = h.in[q] ? v[q] : 0.0;
}

// Every CG kernel solves blockIdx.y = 0 .. nrhs-1 systems at once (the same
// operator, right-hand sides and vectors vs = NP apart, a CGState each); the
// single-system solves are nrhs = 1.
//
// r = b - L phi on free nodes, b = (e/eps0) rho + electrode couplings; electrode
// nodes take their fixed potential (0 when phi_fixed is null: grounded; free
// nodes read the fixed values of their electrode neighbours, so nothing here
// reads what another thread writes); z = D^-1 r; p = 0.  Partials: r.z, r.r, b.b.
__global__ void __launch_bounds__(kThreads)
cg_init_kernel(unsigned NP, int px, int py, int pz, double ipy, double ipz,
               const double* __restrict__ cx,
               const double* __restrict__ cy, const double* __restrict__ cz,
               const double* __restrict__ dinv, const uint8_t* __restrict__ dir,
               const double* __restrict__ phi_fixed, const double* __restrict__ rho,
               double scale, double* phi, double* r, double* zv, double* p, double* partial) {
  const Geo g = geo(px, py, pz, ipy, ipz);
  const long long vo = (long long)blockIdx.y * NP;
  if (rho) rho += vo;
  phi += vo;
  r += vo;
  zv += vo;
  p += vo;
  double acc[3] = {0.0, 0.0, 0.0};
  for (unsigned i = xcd_remap(blockIdx.x, gridDim.x) * kThreads + threadIdx.x; i < NP;
       i += gridDim.x * kThreads) {
    p[i] = 0.0;
    if (dir[i]) {
      phi[i] = phi_fixed ? phi_fixed[i] : 0.0;
      r[i] = 0.0;
      zv[i] = 0.0;
      continue;
    }
    int x, y, z;
    coords(i, g, x, y, z);
    const double ui = phi[i];
    const double f = rho ? scale * rho[i] : 0.0;   // no charge array: rho = 0
    const double lphi = link_sum(i, x, y, z, g, cx, cy, cz, ui, [&](unsigned j) {
      return dir[j] ? (phi_fixed ? phi_fixed[j] : 0.0) : phi[j];
    });
    // electrode couplings of b: sum over electrode neighbours of c phi_fixed
    const double bdir = link_sum(i, x, y, z, g, cx, cy, cz, 0.0, [&](unsigned j) {
      return (dir[j] && phi_fixed) ? -phi_fixed[j] : 0.0;
    });
    const double ri = f - lphi;
    const double zi = dinv[i] * ri;
    r[i] = ri;
    zv[i] = zi;
    const double b = f + bdir;
    acc[0] += ri * zi;
    acc[1] += ri * ri;
    acc[2] += b * b;
  }
  block_sums<3>(acc, partial + 3LL * ((long long)blockIdx.y * gridDim.x + blockIdx.x));
}

__global__ void __launch_bounds__(kRedThreads)
cg_start_kernel(const double* partial, int nblk, double tol, CGState* st) {
  __shared__ double s[3];
  st += blockIdx.y;
  reduce_partials<3>(partial + 3LL * blockIdx.y * nblk, nblk, s);
  if (threadIdx.x == 0) {
    st->rz = s[0];
    st->rr = s[1];
    st->bb = s[2];
    st->thr = tol * tol * s[2];
    st->beta = 0.0;
    st->alpha = 0.0;
    st->it = 0;
    st->breakdown = 0;
    st->done = s[1] <= st->thr ? 1 : 0;
  }
}

// p_new = z + beta p_old (at the node and its neighbours: the old direction is
// not overwritten, p_new goes to the other buffer); q = L p_new; partial p.q
__global__ void __launch_bounds__(kThreads)
cg_matvec_kernel(unsigned NP, int px, int py, int pz, double ipy, double ipz,
                 const double* __restrict__ cx,
                 const double* __restrict__ cy, const double* __restrict__ cz,
                 const uint8_t* __restrict__ dir, const double* __restrict__ zv,
                 const double* __restrict__ p_old, double* __restrict__ p_new,
                 double* __restrict__ q, double* partial, const CGState* st) {
  st += blockIdx.y;
  if (st->done) return;
  const double beta = st->beta;
  const Geo g = geo(px, py, pz, ipy, ipz);
  const long long vo = (long long)blockIdx.y * NP;
  zv += vo;
  p_old += vo;
  p_new += vo;
  q += vo;
  double acc[1] = {0.0};
  for (unsigned i = xcd_remap(blockIdx.x, gridDim.x) * kThreads + threadIdx.x; i < NP;
       i += gridDim.x * kThreads) {
    int x, y, z;
    coords(i, g, x, y, z);
    const Hood h = hood(i, x, y, z, g.px, g.py, g.pz, g.sx, g.sy);
    const bool d = dir[i] != 0;
    double c[6], zn[6], pn[6];
    hood_weights(i, h, cx, cy, cz, c);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      zn[k] = zv[h.j[k]];
      pn[k] = p_old[h.j[k]];
    }
    const double pi = zv[i] + beta * p_old[i];
    // electrode neighbours hold z = p_old = 0, so their p_new is 0 as well
    double qi = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) qi += c[k] * (pi - (zn[k] + beta * pn[k]));
    p_new[i] = d ? 0.0 : pi;
    q[i] = d ? 0.0 : qi;
    acc[0] += d ? 0.0 : pi * qi;
  }
  block_sums<1>(acc, partial + (long long)blockIdx.y * gridDim.x + blockIdx.x);
}

__global__ void __launch_bounds__(kRedThreads)
cg_alpha_kernel(const double* partial, int nblk, CGState* st) {
  st += blockIdx.y;
  if (st->done) return;
  __shared__ double s[1];
  reduce_partials<1>(partial + (long long)blockIdx.y * nblk, nblk, s);
  if (threadIdx.x == 0) {
    if (!(s[0] > 0.0)) {   // the operator is not positive definite on this vector
      st->breakdown = 1;
      st->done = 1;
    } else {
      st->alpha = st->rz / s[0];
    }
  }
}

// phi += alpha p; r -= alpha q; z = D^-1 r (the Jacobi-preconditioned iteration;
// the multigrid one does its update inside the finest restriction); partials r.z, r.r
__global__ void __launch_bounds__(kThreads)
cg_update_kernel(long long NP, const double* __restrict__ dinv, const double* __restrict__ p,
                 const double* __restrict__ q, double* phi, double* r, double* zv,
                 double* partial, const CGState* st) {
  st += blockIdx.y;
  if (st->done) return;
  const double alpha = st->alpha;
  const long long vo = (long long)blockIdx.y * NP;
  p += vo;
  q += vo;
  phi += vo;
  r += vo;
  zv += vo;
  double acc[2] = {0.0, 0.0};
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < NP;
       i += (long long)gridDim.x * kThreads) {
    const double pi = p[i];
    phi[i] += alpha * pi;
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    const double zi = dinv[i] * ri;
    zv[i] = zi;
    acc[0] += ri * zi;
    acc[1] += ri * ri;
  }
  block_sums<2>(acc, partial + 2LL * ((long long)blockIdx.y * gridDim.x + blockIdx.x));
}

__global__ void __launch_bounds__(kRedThreads)
cg_beta_kernel(const double* partial, int nblk, int max_iter, CGState* st) {
  st += blockIdx.y;
  if (st->done) return;
  __shared__ double s[2];
  reduce_partials<2>(partial + 2LL * blockIdx.y * nblk, nblk, s);
  if (threadIdx.x == 0) {
    st->beta = st->rz > 0.0 ? s[0] / st->rz : 0.0;
    st->rz = s[0];
    st->rr = s[1];
    st->it += 1;
    st->done = (s[1] <= st->thr || st->it >= max_iter) ? 1 : 0;
  }
}

// with the multigrid preconditioner: r.z from the V-cycle's partials (nblk_rz per
// system), r.r from the update's (nblk per system)
__global__ void __launch_bounds__(kRedThreads)
cg_beta_mg_kernel(const double* partial, int nblk, const double* partial_rz, int nblk_rz,
                  int max_iter, CGState* st) {
  st += blockIdx.y;
  if (st->done) return;
  __shared__ double s[2], t[1];
  reduce_partials<2>(partial + 2LL * blockIdx.y * nblk, nblk, s);
  reduce_partials<1>(partial_rz + (long long)blockIdx.y * nblk_rz, nblk_rz, t);
  if (threadIdx.x == 0) {
    st->beta = st->rz > 0.0 ? t[0] / st->rz : 0.0;
    st->rz = t[0];
    st->rr = s[1];
    st->it += 1;
    st->done = (s[1] <= st->thr || st->it >= max_iter) ? 1 : 0;
  }
}

// the starting r.z once the V-cycle has replaced the Jacobi z of cg_init
__global__ void __launch_bounds__(kRedThreads)
cg_rz_kernel(const double* partial_rz, int nblk, CGState* st) {
  st += blockIdx.y;
  if (st->done) return;
  __shared__ double t[1];
  reduce_partials<1>(partial_rz + (long long)blockIdx.y * nblk, nblk, t);
  if (threadIdx.x == 0) st->rz = t[0];
}

// ---------------------------------------------------------------------------
// Multigrid preconditioner of the Poisson CG.  On the free nodes the operator is
// A u = diag u - sum_links a u_neighbour (a: free-free link weights; links to an
// electrode only add to diag).  Level k + 1 aggregates 2 x 2 x 2 nodes of level k
// (piecewise-constant prolongation P, restriction P^T): its operator P^T A P keeps
// the same 7-point form, with link weights summed over the aggregates' shared
// faces and diag = sum of the children's diag - 2 (internal link weights).  One
// V-cycle: a damped-Jacobi pre-smoothing from zero (u = w D^-1 b, never stored),
// residual restricted, the coarse problem, the correction prolonged (scaled by
// alpha on the finest level only) and one damped-Jacobi post-smoothing; the
// coarsest level (at most kMGCoarsest nodes) takes an even number of Jacobi
// sweeps.  With w < 2 / lambda_max(D^-1 A) (here <= 2) and alpha < 2 every
// level's cycle is a symmetric positive-definite map, so it preconditions CG.
// ---------------------------------------------------------------------------
struct MGGeo {
  int nx, ny, nz;
  double iny, inz;   // 1 / ny, 1 / nz
};

__device__ __forceinline__ void mg_coords(unsigned i, const MGGeo& g, int& x, int& y, int& z) {
  const unsigned q = udiv(i, (unsigned)g.nz, g.inz);   // x ny + y
  z = (int)(i - q * (unsigned)g.nz);
  x = (int)udiv(q, (unsigned)g.ny, g.iny);
  y = (int)(q - (unsigned)x * (unsigned)g.ny);
}

// level 0: free-free link weights, diagonal and D^-1 of the CG operator
__global__ void __launch_bounds__(kThreads)
mg_level0_kernel(unsigned NP, MGGeo g, const double* __restrict__ cx,
                 const double* __restrict__ cy, const double* __restrict__ cz,
                 const uint8_t* __restrict__ dir, double* ax, double* ay, double* az,
                 double* diag, double* dinv) {
  const unsigned sx = (unsigned)g.ny * g.nz, sy = (unsigned)g.nz;
  for (unsigned i = xcd_remap(blockIdx.x, gridDim.x) * kThreads + threadIdx.x; i < NP; i += gridDim.x * kThreads) {
    int x, y, z;
    mg_coords(i, g, x, y, z);
    const bool f = !dir[i];
    ax[i] = (f && x + 1 < g.nx && !dir[i + sx]) ? cx[i] : 0.0;
    ay[i] = (f && y + 1 < g.ny && !dir[i + sy]) ? cy[i] : 0.0;
    az[i] = (f && z + 1 < g.nz && !dir[i + 1]) ? cz[i] : 0.0;
    double d = 0.0;
    if (f) {
      d = cx[i] + cy[i] + cz[i];
      if (x > 0) d += cx[i - sx];
      if (y > 0) d += cy[i - sy];
      if (z > 0) d += cz[i - 1];
    }
    diag[i] = d;
    dinv[i] = d > 0.0 ? 1.0 / d : 0.0;
  }
}

// level k + 1 from level k (Galerkin with aggregation)
__global__ void __launch_bounds__(kThreads)
mg_coarsen_kernel(MGGeo f, MGGeo c, const double* __restrict__ fax,
                  const double* __restrict__ fay, const double* __restrict__ faz,
                  const double* __restrict__ fdiag, double* cax, double* cay, double* caz,
                  double* cdiag, double* cdinv) {
  const unsigned NC = (unsigned)c.nx * c.ny * c.nz;
  for (unsigned I = xcd_remap(blockIdx.x, gridDim.x) * kThreads + threadIdx.x; I < NC; I += gridDim.x * kThreads) {
    int X, Y, Z;
    mg_coords(I, c, X, Y, Z);
    double d = 0.0, lx = 0.0, ly = 0.0, lz = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int e = 0; e < 2; ++e) {
          const int x = 2 * X + a, y = 2 * Y + b, z = 2 * Z + e;
          if (x >= f.nx || y >= f.ny || z >= f.nz) continue;
          const unsigned j = ((unsigned)x * f.ny + y) * f.nz + z;
          d += fdiag[j];
          if (x + 1 < f.nx) {
            if (a == 0) d -= 2.0 * fax[j];   // link inside the aggregate
            else lx += fax[j];               // link to the next aggregate along x
          }
          if (y + 1 < f.ny) {
            if (b == 0) d -= 2.0 * fay[j];
            else ly += fay[j];
          }
          if (z + 1 < f.nz) {
            if (e == 0) d -= 2.0 * faz[j];
            else lz += faz[j];
          }
        }
    cax[I] = lx;
    cay[I] = ly;
    caz[I] = lz;
    cdiag[I] = d;
    cdinv[I] = d > 0.0 ? 1.0 / d : 0.0;
  }
}

struct MGLevelArgs {
  MGGeo g;
  const double *ax, *ay, *az, *diag, *dinv;
};

__device__ __forceinline__ Hood mg_hood(unsigned j, int x, int y, int z, const MGGeo& g) {
  return hood(j, x, y, z, g.nx, g.ny, g.nz, (unsigned)g.ny * g.nz, (unsigned)g.nz);
}

// (A u)_j with u given by a functor of the neighbour's index and its direction
// (0 .. 5 as in Hood); every load unconditional
template <typename F>
__device__ __forceinline__ double mg_apply(unsigned j, const Hood& h, const MGLevelArgs& L,
                                           double uj, F u) {
  double c[6], v[6];
  hood_weights(j, h, L.ax, L.ay, L.az, c);
#pragma unroll
  for (int k = 0; k < 6; ++k) v[k] = u(h.j[k], k);
  double s = L.diag[j] * uj;
#pragma unroll
  for (int k = 0; k < 6; ++k) s -= c[k] * v[k];
  return s;
}

// b_c[I] = sum over the children j of I of (b - A u)_j, u = w D^-1 b (pre-smoothing).
// Eight consecutive lanes take the eight children of one coarse node (lane bits
// 2, 1, 0 = x, y, z offsets) and sum them by shuffles, so the fine level runs one
// node per thread.  Like the other level kernels it gives every XCD a contiguous
// run of nodes (the x- and y-neighbours a node reads are then in that XCD's L2).
//
// UPD (the finest level inside a CG iteration): the CG update comes first, in the
// same pass -- phi += alpha p and the new residual b - alpha q (b: the old residual),
// formed wherever it is needed (at the node, and at its neighbours from their old b
// and q) and stored to r_new, another buffer, with partial sums (0, r_new.r_new) per
// workgroup -- and the restriction takes the new residual as its right-hand side.
template <bool UPD>
__global__ void __launch_bounds__(kThreads)
mg_restrict_kernel(MGLevelArgs L, MGGeo c, double w, const double* __restrict__ b,
                   long long b_stride, double* bc, long long bc_stride, const CGState* st,
                   const double* __restrict__ p, const double* __restrict__ q,
                   double* __restrict__ phi, double* __restrict__ r_new,
                   double* __restrict__ partial) {
  if (st[blockIdx.y].done) return;
  const double alpha = UPD ? st[blockIdx.y].alpha : 0.0;
  b += blockIdx.y * b_stride;
  bc += blockIdx.y * bc_stride;
  if (UPD) {
    p += blockIdx.y * b_stride;
    q += blockIdx.y * b_stride;
    phi += blockIdx.y * b_stride;
    r_new += blockIdx.y * b_stride;
  }
  const unsigned NC = (unsigned)c.nx * c.ny * c.nz;
  auto rhs = [&](unsigned j) { return UPD ? b[j] - alpha * q[j] : b[j]; };
  auto u = [&](unsigned j, int) { return w * L.dinv[j] * rhs(j); };
  const unsigned ch = threadIdx.x & 7;
  double acc[2] = {0.0, 0.0};
  // trip counts are equal within each group of eight lanes (8 NC and the stride are
  // multiples of eight), so every shuffle below sees its whole group
  for (unsigned t = xcd_remap(blockIdx.x, gridDim.x) * kThreads + threadIdx.x; t < 8 * NC; t += gridDim.x * kThreads) {
    const unsigned I = t >> 3;
    int X, Y, Z;
    mg_coords(I, c, X, Y, Z);
    const int x = 2 * X + (int)(ch >> 2), y = 2 * Y + (int)((ch >> 1) & 1),
              z = 2 * Z + (int)(ch & 1);
    // a child past a ragged edge of the box stands in for the aggregate's first
    // child (which always exists) and contributes nothing
    const bool inb = x < L.g.nx && y < L.g.ny && z < L.g.nz;
    const int xx = inb ? x : 2 * X, yy = inb ? y : 2 * Y, zz = inb ? z : 2 * Z;
    const unsigned j = ((unsigned)xx * L.g.ny + yy) * L.g.nz + zz;
    const double bj = rhs(j);
    const double dj = L.dinv[j];
    const double sj = bj - mg_apply(j, mg_hood(j, xx, yy, zz, L.g), L, w * dj * bj, u);
    double s = (inb && dj != 0.0) ? sj : 0.0;   // active nodes only
    if (UPD && inb) {
      phi[j] += alpha * p[j];
      r_new[j] = bj;
      acc[1] += bj * bj;
    }
    s += __shfl_xor(s, 1, 8);
    s += __shfl_xor(s, 2, 8);
    s += __shfl_xor(s, 4, 8);
    if (ch == 0) bc[I] = s;
  }
  if (UPD) block_sums<2>(acc, partial + 2LL * ((long long)blockIdx.y * gridDim.x + blockIdx.x));
}

// The coarse tail of the V-cycle: levels t .. t + nt - 1 (the last one the
// coarsest), each of at most kMGTailNodes nodes, for one system per workgroup of
// kMGTailNodes threads.  Thread j keeps node j's row of every tail level in
// registers (loaded once) and the vectors live in LDS, so the steps below touch
// memory only to read b_t and write u_t: restriction of the pre-smoothed residual
// level by level, the coarsest level's (even number of) damped-Jacobi sweeps from
// zero, and the corrections back up (prolonged coarse iterate plus w D^-1 b, then
// one damped-Jacobi sweep) -- what the per-level kernels do on the finer levels.
struct MGTailArgs {
  int t, nt;
  MGLevelArgs lv[kMGTailLevels];
};

// node j's row: diagonal, w D^-1, the six link weights (0 past the box or for an
// inactive link) with the neighbours' indices (j itself where the weight is 0),
// and the index of its aggregate on the next coarser level
struct MGRow {
  double dg, wd, a[6];
  unsigned nb[6], parent;
  bool on;
};

__device__ __forceinline__ MGRow mg_row(const MGLevelArgs& A, const MGGeo* c, unsigned j,
                                        double w) {
  MGRow r;
  const unsigned n = (unsigned)A.g.nx * A.g.ny * A.g.nz;
  r.on = j < n;
  r.dg = 0.0;
  r.wd = 0.0;
  r.parent = 0;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    r.a[q] = 0.0;
    r.nb[q] = j;
  }
  if (!r.on) return r;
  int x, y, z;
  mg_coords(j, A.g, x, y, z);
  const unsigned sx = (unsigned)A.g.ny * A.g.nz, sy = (unsigned)A.g.nz;
  if (x + 1 < A.g.nx) { r.a[0] = A.ax[j]; r.nb[0] = j + sx; }
  if (x > 0) { r.a[1] = A.ax[j - sx]; r.nb[1] = j - sx; }
  if (y + 1 < A.g.ny) { r.a[2] = A.ay[j]; r.nb[2] = j + sy; }
  if (y > 0) { r.a[3] = A.ay[j - sy]; r.nb[3] = j - sy; }
  if (z + 1 < A.g.nz) { r.a[4] = A.az[j]; r.nb[4] = j + 1; }
  if (z > 0) { r.a[5] = A.az[j - 1]; r.nb[5] = j - 1; }
  r.dg = A.diag[j];
  r.wd = w * A.dinv[j];
  if (c)
    r.parent = (unsigned)(x >> 1) * ((unsigned)c->ny * c->nz) + (unsigned)(y >> 1) * c->nz +
               (unsigned)(z >> 1);
  return r;
}

// (A u)_j, the row's order of terms as in mg_apply
__device__ __forceinline__ double mg_row_apply(const MGRow& r, const double* u, double uj) {
  double s = r.dg * uj;
#pragma unroll
  for (int q = 0; q < 6; ++q) s -= r.a[q] * u[r.nb[q]];
  return s;
}

__global__ void __launch_bounds__(kMGTailNodes)
mg_tail_kernel(MGTailArgs T, double w, int sweeps, const double* __restrict__ bt,
               double* __restrict__ ut, long long v_stride, const CGState* st) {
  if (st[blockIdx.y].done) return;
  bt += blockIdx.y * v_stride;
  ut += blockIdx.y * v_stride;
  // per level b and u, the coarsest level's second iterate, the residual scratch
  __shared__ double sb[kMGTailLevels][kMGTailNodes], su[kMGTailLevels][kMGTailNodes];
  __shared__ double su2[kMGTailNodes], sr[kMGTailNodes];
  const unsigned j = threadIdx.x;
  const int nt = T.nt;
  MGRow row[kMGTailLevels];
#pragma unroll
  for (int s = 0; s < kMGTailLevels; ++s) {
    row[s] = mg_row(T.lv[s], s + 1 < nt ? &T.lv[s + 1].g : nullptr, j, w);
    row[s].on = row[s].on && s < nt;
  }
  if (row[0].on) sb[0][j] = bt[j];
  __syncthreads();
#pragma unroll
  for (int s = 0; s + 1 < kMGTailLevels; ++s) {   // restriction s -> s + 1
    if (s + 1 >= nt) break;
    if (row[s].on) su[s][j] = row[s].wd * sb[s][j];
    __syncthreads();
    if (row[s].on)
      sr[j] = row[s].wd != 0.0 ? sb[s][j] - mg_row_apply(row[s], su[s], su[s][j]) : 0.0;
    __syncthreads();
    if (row[s + 1].on) {   // sum over the children of this aggregate
      const MGGeo& f = T.lv[s].g;
      int X, Y, Z;
      mg_coords(j, T.lv[s + 1].g, X, Y, Z);
      double acc = 0.0;
      for (int ch = 0; ch < 8; ++ch) {
        const int x = 2 * X + (ch >> 2), y = 2 * Y + ((ch >> 1) & 1), z = 2 * Z + (ch & 1);
        if (x < f.nx && y < f.ny && z < f.nz) acc += sr[((unsigned)x * f.ny + y) * f.nz + z];
      }
      sb[s + 1][j] = acc;
    }
    __syncthreads();
  }
  // the coarsest level: sweeps from zero, ping-pong between su[c] and su2
  const int c = nt - 1;
  MGRow rc = row[0];
  const double* bc = sb[0];
  double* u0 = su[0];
#pragma unroll
  for (int s = 1; s < kMGTailLevels; ++s)
    if (s == c) {
      rc = row[s];
      bc = sb[s];
      u0 = su[s];
    }
  if (rc.on) u0[j] = 0.0;
  __syncthreads();
  for (int q = 0; q < sweeps; ++q) {
    const double* uo = (q & 1) ? su2 : u0;
    double* un = (q & 1) ? u0 : su2;
    if (rc.on) {
      const double uj = uo[j];
      un[j] = uj + rc.wd * (bc[j] - mg_row_apply(rc, uo, uj));
    }
    __syncthreads();
  }
  if (nt == 1) {   // sweeps is even: the result is in u0
    if (rc.on) ut[j] = u0[j];
    return;
  }
#pragma unroll
  for (int s = kMGTailLevels - 2; s >= 0; --s) {   // correction of s from s + 1
    if (s + 1 >= nt) continue;
    const double* E = (s + 1 == c) ? su[s + 1] : sb[s + 1];   // level s + 1's result
    if (row[s].on)
      su[s][j] = row[s].wd == 0.0 ? 0.0 : row[s].wd * sb[s][j] + E[row[s].parent];
    __syncthreads();
    if (row[s].on) {
      const double uj = su[s][j];
      const double o =
          row[s].wd == 0.0 ? 0.0 : uj + row[s].wd * (sb[s][j] - mg_row_apply(row[s], su[s], uj));
      if (s > 0) sb[s][j] = o;
      else ut[j] = o;
    }
    __syncthreads();
  }
}

// u' = w D^-1 b + alpha P e (the pre-smoothed u plus the prolonged correction),
// then one damped-Jacobi sweep: out = u' + w D^-1 (b - A u').  On level 0, out is
// the CG's z and the partial sums of r.z go to partial_rz.
template <bool FINEST>
__global__ void __launch_bounds__(kThreads)
mg_correct_kernel(MGLevelArgs L, MGGeo c, double w, double alpha, const double* __restrict__ b,
                  long long b_stride, const double* __restrict__ e, long long e_stride,
                  double* out, long long out_stride, double* partial_rz, const CGState* st) {
  if (st[blockIdx.y].done) return;
  b += blockIdx.y * b_stride;
  e += blockIdx.y * e_stride;
  out += blockIdx.y * out_stride;
  const unsigned N = (unsigned)L.g.nx * L.g.ny * L.g.nz;
  const unsigned sxc = (unsigned)c.ny * c.nz;
  auto parent = [&](int x, int y, int z) {
    return (unsigned)(x >> 1) * sxc + (unsigned)(y >> 1) * c.nz + (unsigned)(z >> 1);
  };
  double acc[1] = {0.0};
  for (unsigned j = xcd_remap(blockIdx.x, gridDim.x) * kThreads + threadIdx.x; j < N; j += gridDim.x * kThreads) {
    int x, y, z;
    mg_coords(j, L.g, x, y, z);
    const Hood h = mg_hood(j, x, y, z, L.g);
    // the node and its six neighbours (a clamped one is j itself, weight 0): D^-1, b
    // and the coarse correction of the aggregate, all loaded before any is used
    double dv[7], bv[7], ev[7], c[6];
    {
      unsigned m[7], P[7];
      m[6] = j;
      P[6] = parent(x, y, z);
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const int dx = (k == 0) - (k == 1), dy = (k == 2) - (k == 3), dz = (k == 4) - (k == 5);
        m[k] = h.j[k];
        P[k] = h.in[k] ? parent(x + dx, y + dy, z + dz) : P[6];
      }
      hood_weights(j, h, L.ax, L.ay, L.az, c);
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        dv[k] = L.dinv[m[k]];
        bv[k] = b[m[k]];
        ev[k] = e[P[k]];
      }
    }
    // u' = w D^-1 b + alpha P e on active nodes, 0 elsewhere
    double u[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) u[k] = dv[k] == 0.0 ? 0.0 : w * dv[k] * bv[k] + alpha * ev[k];
    double au = L.diag[j] * u[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) au -= c[k] * u[k];
    const double o = dv[6] == 0.0 ? 0.0 : u[6] + w * dv[6] * (bv[6] - au);
    out[j] = o;
    if (FINEST) acc[0] += bv[6] * o;
  }
  if (FINEST) block_sums<1>(acc, partial_rz + (long long)blockIdx.y * gridDim.x + blockIdx.x);
}

// ---------------------------------------------------------------------------
// occupancy, density, potential on the Schroedinger grid
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// one wave; lane j holds state j (nev <= 64).  f = 1 / (1 + exp((E - mu) / kT))
// written as (1 - tanh((E - mu) / 2kT)) / 2; mu by bisection on sum f = n_holes.
__global__ void __launch_bounds__(64)
occupancy_kernel(int nev, const double* __restrict__ E, double n_holes, double kT, double* f,
                 double* mu_out) {
  const int j = threadIdx.x;
  const bool has = j < nev;
  const double e = has ? E[j] : 0.0;
  double lo = wave_min(has ? e : 1e300) - 60.0 * kT - 1.0;
  double hi = wave_max(has ? e : -1e300) + 60.0 * kT + 1.0;
  const double inv2kT = 0.5 / kT;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    const double s = wave_sum(has ? 0.5 * (1.0 - tanh((e - mid) * inv2kT)) : 0.0);
    if (s > n_holes) hi = mid; else lo = mid;
  }
  const double mu = 0.5 * (lo + hi);
  if (has) f[j] = 0.5 * (1.0 - tanh((e - mu) * inv2kT));
  if (j == 0 && mu_out) *mu_out = mu;
}

// rho (P grid) = rho_fixed + embedded hole density; density (S grid) =
// sum_n f_n sum_c |psi_n,c|^2 / h^3 with psi [nev][nx][ny][nz][6] (vector
// stride vstride complex entries)
__global__ void __launch_bounds__(kThreads)
rho_kernel(unsigned NP, int px, int py, int pz, double ipy, double ipz, int ox, int oy, int oz,
           int nx, int ny, int nz,
           int nev, const double2* __restrict__ psi, long long vstride,
           const double* __restrict__ f, double inv_h3, const double* __restrict__ rho_fixed,
           double* rho, double* density) {
  const Geo g = geo(px, py, pz, ipy, ipz);
  for (unsigned i = xcd_remap(blockIdx.x, gridDim.x) * kThreads + threadIdx.x; i < NP;
       i += gridDim.x * kThreads) {
    int x, y, z;
    coords(i, g, x, y, z);
    x -= ox;
    y -= oy;
    z -= oz;
    double v = rho_fixed ? rho_fixed[i] : 0.0;
    if (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz) {
      const long long s = ((long long)x * ny + y) * nz + z;
      double d = 0.0;
      for (int n = 0; n < nev; ++n) {
        const double2* q = psi + n * vstride + 6 * s;
        double a = 0.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) a += q[c].x * q[c].x + q[c].y * q[c].y;
        d += f[n] * a;
      }
      d *= inv_h3;
      v += d;
      if (density) density[s] = d;
    }
    if (rho) rho[i] = v;
  }
}

// V (S grid) = V_off + phi at the embedded nodes
__global__ void __launch_bounds__(kThreads)
extract_kernel(long long NS, int nx, int ny, int nz, int py, int pz, int ox, int oy, int oz,
               const double* __restrict__ V_off, const double* __restrict__ phi, double* V) {
  for (long long s = (long long)blockIdx.x * kThreads + threadIdx.x; s < NS;
       s += (long long)gridDim.x * kThreads) {
    const int x = (int)(s / ((long long)ny * nz)), y = (int)((s / nz) % ny), z = (int)(s % nz);
    V[s] = V_off[s] + phi[((long long)(x + ox) * py + (y + oy)) * pz + (z + oz)];
  }
}

// ---------------------------------------------------------------------------
// Anderson mixing
// ---------------------------------------------------------------------------
// F = phi_out - phi_in; partial max |F|
__global__ void __launch_bounds__(kThreads)
residual_kernel(long long NP, const double* __restrict__ phi_in,
                const double* __restrict__ phi_out, double* F, double* partial) {
  double m = 0.0;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < NP;
       i += (long long)gridDim.x * kThreads) {
    const double d = phi_out[i] - phi_in[i];
    F[i] = d;
    m = fmax(m, fabs(d));
  }
  __shared__ double sh[kThreads / 64];
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int k = 0; k < kThreads / 64; ++k) r = fmax(r, sh[k]);
    partial[blockIdx.x] = r;
  }
}

__global__ void __launch_bounds__(kThreads)
max_reduce_kernel(const double* partial, int nblk, double* out) {
  double m = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kThreads) m = fmax(m, partial[b]);
  __shared__ double sh[kThreads / 64];
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int k = 0; k < kThreads / 64; ++k) r = fmax(r, sh[k]);
    *out = r;
  }
}

// partials of F.F and F.F_j for the k stored residuals (slots listed in order)
template <int K>
__global__ void __launch_bounds__(kThreads)
anderson_dots_kernel(long long NP, const double* __restrict__ F,
                     const double* __restrict__ histF, double* partial) {
  double acc[K + 1];
#pragma unroll
  for (int j = 0; j <= K; ++j) acc[j] = 0.0;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < NP;
       i += (long long)gridDim.x * kThreads) {
    const double fi = F[i];
    acc[0] += fi * fi;
#pragma unroll
    for (int j = 0; j < K; ++j) acc[j + 1] += fi * histF[(long long)j * NP + i];
  }
  block_sums<K + 1>(acc, partial + (long long)(K + 1) * blockIdx.x);
}

template <int K>
__global__ void __launch_bounds__(kRedThreads)
anderson_dots_reduce_kernel(const double* partial, int nblk, double* dots) {
  __shared__ double s[K + 1];
  reduce_partials<K + 1>(partial, nblk, s);
  __syncthreads();
  if (threadIdx.x <= K) dots[threadIdx.x] = s[threadIdx.x];
}

// Least squares over the k stored (x_j, F_j): minimise |F - sum_j g_j (F - F_j)|
// through the normal equations (k <= 8, a relative 1e-12 ridge keeps them
// solvable when two stored residuals nearly coincide); then record the new
// entry's row of the stored Gram matrix G[j][l] = F_j . F_l at `slot`.
__global__ void anderson_coef_kernel(int k, int m, int slot, const double* __restrict__ dots,
                                     double* G, double* gamma) {
  if (threadIdx.x != 0) return;
  const double FF = dots[0];
  double A[8][9];
  for (int j = 0; j < k; ++j) {
    for (int l = 0; l < k; ++l)
      A[j][l] = FF - dots[1 + j] - dots[1 + l] + G[j * m + l];
    A[j][k] = FF - dots[1 + j];
  }
  double tr = 0.0;
  for (int j = 0; j < k; ++j) tr += A[j][j];
  const double ridge = 1e-12 * (tr > 0.0 ? tr / (k > 0 ? k : 1) : 1.0);
  for (int j = 0; j < k; ++j) A[j][j] += ridge;
  // Gaussian elimination with partial pivoting
  for (int c = 0; c < k; ++c) {
    int piv = c;
    for (int r = c + 1; r < k; ++r)
      if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
    if (piv != c)
      for (int l = 0; l <= k; ++l) {
        const double t = A[c][l];
        A[c][l] = A[piv][l];
        A[piv][l] = t;
      }
    const double d = A[c][c];
    for (int r = c + 1; r < k; ++r) {
      const double fct = d != 0.0 ? A[r][c] / d : 0.0;
      for (int l = c; l <= k; ++l) A[r][l] -= fct * A[c][l];
    }
  }
  for (int c = k - 1; c >= 0; --c) {
    double s = A[c][k];
    for (int l = c + 1; l < k; ++l) s -= A[c][l] * gamma[l];
    gamma[c] = A[c][c] != 0.0 ? s / A[c][c] : 0.0;
  }
  // the new entry (current x, F) replaces `slot`; its dots with the other
  // stored residuals are the ones just computed (slot j holds stored entry j)
  for (int j = 0; j < m; ++j) {
    if (j == slot) continue;
    if (j < k) {
      G[slot * m + j] = dots[1 + j];
      G[j * m + slot] = dots[1 + j];
    }
  }
  G[slot * m + slot] = FF;
}

// x <- x + a F - sum_j g_j ((x - x_j) + a (F - F_j)); the current (x, F) is
// then stored in `slot` (after every stored entry has been read at this node)
template <int K>
__global__ void __launch_bounds__(kThreads)
anderson_update_kernel(long long NP, int slot, double a, const double* __restrict__ gamma,
                       double* x, const double* __restrict__ F, double* histX, double* histF) {
  double g[K > 0 ? K : 1];
#pragma unroll
  for (int j = 0; j < K; ++j) g[j] = gamma[j];
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < NP;
       i += (long long)gridDim.x * kThreads) {
    const double xi = x[i], fi = F[i];
    double v = xi + a * fi;
#pragma unroll
    for (int j = 0; j < K; ++j)
      v -= g[j] * ((xi - histX[(long long)j * NP + i]) + a * (fi - histF[(long long)j * NP + i]));
    if (slot >= 0) {
      histX[(long long)slot * NP + i] = xi;
      histF[(long long)slot * NP + i] = fi;
    }
    x[i] = v;
  }
}

// ---------------------------------------------------------------------------
// configuration interaction: pair densities, their potentials, integrals
// ---------------------------------------------------------------------------
// (j, l), j <= l, of pair q in lexicographic order over M orbitals
__device__ __forceinline__ void pair_of(int q, int M, int& j, int& l) {
  j = 0;
  while (q >= M - j) {
    q -= M - j;
    ++j;
  }
  l = j + q;
}

// right-hand sides 2q (real part) and 2q+1 (imaginary part) of pair q:
// rho_jl = sum_b conj(phi_j,b) phi_l,b / h^3 at the embedded nodes, 0 elsewhere
__global__ void __launch_bounds__(kThreads)
pair_rhs_kernel(unsigned NP, int px, int py, int pz, double ipy, double ipz, int ox, int oy,
                int oz, int nx, int ny, int nz, int M, const double2* __restrict__ phi,
                double inv_h3, double* rhs) {
  const Geo g = geo(px, py, pz, ipy, ipz);
  int j, l;
  pair_of(blockIdx.y, M, j, l);
  const long long NS = (long long)nx * ny * nz;
  double* re = rhs + 2LL * blockIdx.y * NP;
  double* im = re + NP;
  for (unsigned i = blockIdx.x * kThreads + threadIdx.x; i < NP; i += gridDim.x * kThreads) {
    int x, y, z;
    coords(i, g, x, y, z);
    x -= ox;
    y -= oy;
    z -= oz;
    double a = 0.0, b = 0.0;
    if (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz) {
      const long long s = ((long long)x * ny + y) * nz + z;
      const double2* pj = phi + ((long long)j * NS + s) * 3;
      const double2* pl = phi + ((long long)l * NS + s) * 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) {   // conj(pj) * pl
        a += pj[c].x * pl[c].x + pj[c].y * pl[c].y;
        b += pj[c].x * pl[c].y - pj[c].y * pl[c].x;
      }
    }
    re[i] = a * inv_h3;
    // a self pair density is real; with contracted multiply-adds the sum above
    // leaves rounding noise there, which the solver would chase to tolerance
    im[i] = j == l ? 0.0 : b * inv_h3;
  }
}

// Vc[q][s] = V[2q] + i V[2q+1] at the Schroedinger-grid nodes
__global__ void __launch_bounds__(kThreads)
pair_potential_gather_kernel(long long NS, int nx, int ny, int nz, long long NP, int py, int pz,
                             int ox, int oy, int oz, const double* __restrict__ V, double2* Vc) {
  const long long s = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (s >= NS) return;
  const int q = blockIdx.y;
  const int x = (int)(s / ((long long)ny * nz)), y = (int)((s / nz) % ny), z = (int)(s % nz);
  const long long i = ((long long)(x + ox) * py + (y + oy)) * pz + (z + oz);
  Vc[(long long)q * NS + s] = make_double2(V[2LL * q * NP + i], V[(2LL * q + 1) * NP + i]);
}

// A[(i, k)][s] = sum_b phi_i,b conj(phi_k,b) (so that conj(A) is the pair product)
__global__ void __launch_bounds__(kThreads)
pair_product_kernel(long long NS, int M, const double2* __restrict__ phi, double2* A) {
  const long long s = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (s >= NS) return;
  const int i = blockIdx.y / M, k = blockIdx.y % M;
  const double2* pi = phi + ((long long)i * NS + s) * 3;
  const double2* pk = phi + ((long long)k * NS + s) * 3;
  double a = 0.0, b = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {   // pi * conj(pk)
    a += pi[c].x * pk[c].x + pi[c].y * pk[c].y;
    b += pi[c].y * pk[c].x - pi[c].x * pk[c].y;
  }
  A[(long long)blockIdx.y * NS + s] = make_double2(a, b);
}

// (ik|jl) from the stored pairs: Cs[(i, k)][q(j, l)] for j <= l, else
// conj(Cs[(k, i)][q(l, j)]) (V_lj = conj(V_jl), conj(rho_ik) = rho_ki)
__device__ double2 coulomb(const double2* Cs, int M, int P, int i, int k, int j, int l) {
  if (j <= l) {
    const int q = j * M - j * (j - 1) / 2 + (l - j);
    return Cs[(long long)(i * M + k) * P + q];
  }
  const int q = l * M - l * (l - 1) / 2 + (j - l);
  const double2 c = Cs[(long long)(k * M + i) * P + q];
  return make_double2(c.x, -c.y);
}

// determinant a -> (u, v), u < v, lexicographic over n spin-orbitals
__device__ void det_of(int a, int n, int& u, int& v) {
  u = 0;
  while (a >= n - 1 - u) {
    a -= n - 1 - u;
    ++u;
  }
  v = u + 1 + a;
}

__device__ double2 two_body(const double2* Cs, int M, int P, int u, int v, int w, int x) {
  if ((u & 1) != (w & 1) || (v & 1) != (x & 1)) return make_double2(0.0, 0.0);
  return coulomb(Cs, M, P, u >> 1, w >> 1, v >> 1, x >> 1);
}

// H[a][b] = h_uw d_vx + h_vx d_uw - h_ux d_vw - h_vw d_ux + <uv|wx> - <uv|xw>
__global__ void __launch_bounds__(kThreads)
ci_assemble_kernel(int M, int P, const double2* __restrict__ hsp, const double2* __restrict__ Cs,
                   double2* H) {
  const int n = 2 * M, K = n * (n - 1) / 2;
  const int idx = blockIdx.x * kThreads + threadIdx.x;
  if (idx >= K * K) return;
  const int a = idx / K, b = idx % K;
  int u, v, w, x;
  det_of(a, n, u, v);
  det_of(b, n, w, x);
  double2 acc = make_double2(0.0, 0.0);
  auto add = [&](double2 t, double sgn) {
    acc.x += sgn * t.x;
    acc.y += sgn * t.y;
  };
  if (v == x) add(hsp[u * n + w], 1.0);
  if (u == w) add(hsp[v * n + x], 1.0);
  if (v == w) add(hsp[u * n + x], -1.0);
  if (u == x) add(hsp[v * n + w], -1.0);
  add(two_body(Cs, M, P, u, v, w, x), 1.0);
  add(two_body(Cs, M, P, u, v, x, w), -1.0);
  H[idx] = acc;
}

// full tensor (ik|jl), [M][M][M][M] complex
__global__ void __launch_bounds__(kThreads)
coulomb_expand_kernel(int M, int P, const double2* __restrict__ Cs, double2* C) {
  const int idx = blockIdx.x * kThreads + threadIdx.x;
  if (idx >= M * M * M * M) return;
  const int i = idx / (M * M * M), k = (idx / (M * M)) % M, j = (idx / M) % M, l = idx % M;
  C[idx] = coulomb(Cs, M, P, i, k, j, l);
}

// J = mean(E_1, E_2, E_3) - E_0 of the ascending two-hole spectrum
__global__ void exchange_kernel(const double* E, double* J) {
  if (threadIdx.x == 0) J[0] = (E[1] + E[2] + E[3]) / 3.0 - E[0];
}

__global__ void __launch_bounds__(kRedThreads)
sum1_kernel(const double* partial, int nblk, double* out) {
  __shared__ double s[1];
  reduce_partials<1>(partial, nblk, s);
  if (threadIdx.x == 0) *out = s[0];
}

template <int K>
void anderson_k(const PGeom& g, int nb, int m, int slot, double mixing, double* x,
                const double* F, double* histX, double* histF, double* G, double* dots,
                double* gamma, double* partial, hipStream_t s) {
  if (m > 0) {
    anderson_dots_kernel<K><<<nb, kThreads, 0, s>>>(g.NP, F, histF, partial);
    anderson_dots_reduce_kernel<K><<<1, kRedThreads, 0, s>>>(partial, nb, dots);
    anderson_coef_kernel<<<1, 64, 0, s>>>(K, m, slot, dots, G, gamma);
  }
  anderson_update_kernel<K><<<nb, kThreads, 0, s>>>(g.NP, m > 0 ? slot : -1, mixing, gamma, x,
                                                     F, histX, histF);
}

}  // namespace

int sp_blocks(long long n) {
  const long long b = (n + kThreads - 1) / kThreads;
  return (int)(b < kRedBlocks ? (b > 0 ? b : 1) : kRedBlocks);
}

size_t sp_partial_doubles(int nrhs) { return (size_t)kRedBlocks * 9 * (nrhs > 0 ? nrhs : 1); }

hipError_t launch_pcoef(const PGeom& g, double h, const double* eps, const uint8_t* dir,
                        double* cx, double* cy, double* cz, double* dinv, double* partial,
                        double* n_dir, hipStream_t s) {
  const int nb = sp_blocks(g.NP);
  pcoef_kernel<<<nb, kThreads, 0, s>>>((unsigned)g.NP, g.px, g.py, g.pz, 1.0 / g.py, 1.0 / g.pz,
                                       1.0 / (h * h), eps, dir, cx, cy, cz, dinv, partial);
  sum1_kernel<<<1, kRedThreads, 0, s>>>(partial, nb, n_dir);
  return hipGetLastError();
}

hipError_t launch_cg_init(const PGeom& g, const double* cx, const double* cy, const double* cz,
                          const double* dinv, const uint8_t* dir, const double* phi_fixed,
                          const double* rho, double scale, double* phi, double* r, double* z,
                          double* p, double* partial, double tol, CGState* st, hipStream_t s,
                          int nrhs) {
  const int nb = sp_blocks(g.NP);
  cg_init_kernel<<<dim3(nb, nrhs), kThreads, 0, s>>>((unsigned)g.NP, g.px, g.py, g.pz, 1.0 / g.py,
                                         1.0 / g.pz, cx, cy, cz, dinv, dir, phi_fixed, rho,
                                         scale, phi, r, z, p, partial);
  cg_start_kernel<<<dim3(1, nrhs), kRedThreads, 0, s>>>(partial, nb, tol, st);
  return hipGetLastError();
}

namespace {
MGGeo mg_geo(const MGLevel& L) { return MGGeo{L.nx, L.ny, L.nz, 1.0 / L.ny, 1.0 / L.nz}; }
MGLevelArgs mg_args(const MGData& m, int k) {
  const MGLevel& L = m.plan.lv[k];
  return MGLevelArgs{mg_geo(L), m.ax + L.off, m.ay + L.off, m.az + L.off, m.diag + L.off,
                     m.dinv + L.off};
}
}  // namespace

hipError_t launch_mg_vcycle(const PGeom& g, const MGData& m, const double* r, double* z,
                            const CGState* st, int nrhs, hipStream_t s, bool restrict0);

hipError_t launch_cg_iter(const PGeom& g, const double* cx, const double* cy, const double* cz,
                          const double* dinv, const uint8_t* dir, double* z,
                          const double* p_old, double* p_new, double* q, double* phi,
                          double* r, double* partial, int max_iter, CGState* st,
                          hipStream_t s, int nrhs, const MGData* mg) {
  const int nb = sp_blocks(g.NP);
  cg_matvec_kernel<<<dim3(nb, nrhs), kThreads, 0, s>>>((unsigned)g.NP, g.px, g.py, g.pz, 1.0 / g.py,
                                           1.0 / g.pz, cx, cy, cz, dir, z, p_old, p_new, q,
                                           partial, st);
  cg_alpha_kernel<<<dim3(1, nrhs), kRedThreads, 0, s>>>(partial, nb, st);
  if (!mg) {
    cg_update_kernel<<<dim3(nb, nrhs), kThreads, 0, s>>>(g.NP, dinv, p_new, q, phi, r, z,
                                                               partial, st);
    cg_beta_kernel<<<dim3(1, nrhs), kRedThreads, 0, s>>>(partial, nb, max_iter, st);
    return hipGetLastError();
  }
  // the update inside the finest restriction: the new r goes to z's buffer (z is
  // spent once p_new is formed) and the V-cycle's z to r's, so the caller swaps the
  // two buffers from one iteration to the next
  const MGPlan& P = mg->plan;
  const unsigned nbu = (unsigned)sp_blocks(8 * P.lv[1].N);
  mg_restrict_kernel<true><<<dim3(nbu, nrhs), kThreads, 0, s>>>(
      mg_args(*mg, 0), mg_geo(P.lv[1]), kMGOmega, r, g.NP, mg->b + P.lv[1].voff, P.vtotal, st,
      p_new, q, phi, z, partial);
  const hipError_t e = launch_mg_vcycle(g, *mg, z, r, st, nrhs, s, false);
  if (e != hipSuccess) return e;
  cg_beta_mg_kernel<<<dim3(1, nrhs), kRedThreads, 0, s>>>(partial, (int)nbu, mg->partial_rz, nb,
                                                          max_iter, st);
  return hipGetLastError();
}

MGPlan mg_plan(const PGeom& g) {
  MGPlan P{};
  int nx = g.px, ny = g.py, nz = g.pz;
  long long off = 0, voff = 0;
  for (int k = 0; k < kMGMaxLevels; ++k) {
    MGLevel& L = P.lv[k];
    L.nx = nx;
    L.ny = ny;
    L.nz = nz;
    L.N = (long long)nx * ny * nz;
    L.off = off;
    L.voff = k == 0 ? 0 : voff;
    off += L.N;
    if (k > 0) voff += L.N;
    P.nlev = k + 1;
    if ((k > 0 && L.N <= kMGCoarsest) || (nx == 1 && ny == 1 && nz == 1 && k > 0)) break;
    nx = (nx + 1) / 2;
    ny = (ny + 1) / 2;
    nz = (nz + 1) / 2;
  }
  P.total = off;
  P.vtotal = voff;
  // the tail: the levels of at most kMGTailNodes nodes, at most kMGTailLevels of
  // them, never level 0 (level sizes do not grow towards the coarsest)
  const int L = P.nlev - 1;
  P.tail = L;
  while (P.tail > 1 && P.tail > L - kMGTailLevels + 1 && P.lv[P.tail - 1].N <= kMGTailNodes)
    --P.tail;
  return P;
}

namespace {
MGGeo mgeo(const MGLevel& L) { return mg_geo(L); }
MGLevelArgs margs(const MGData& m, int k) { return mg_args(m, k); }
unsigned mg_blocks(long long n) { return (unsigned)sp_blocks(n); }
}  // namespace

hipError_t launch_mg_setup(const PGeom& g, const double* cx, const double* cy, const double* cz,
                           const uint8_t* dir, const MGData& m, hipStream_t s) {
  const MGPlan& P = m.plan;
  if (P.lv[P.nlev - 1].N > kMGCoarsest || P.nlev < 2 || P.tail < 1 || P.tail >= P.nlev ||
      P.nlev - P.tail > kMGTailLevels || P.lv[P.tail].N > kMGTailNodes)
    return hipErrorInvalidValue;
  mg_level0_kernel<<<mg_blocks(g.NP), kThreads, 0, s>>>((unsigned)g.NP, mgeo(P.lv[0]), cx, cy,
                                                        cz, dir, m.ax, m.ay, m.az, m.diag,
                                                        m.dinv);
  for (int k = 0; k + 1 < P.nlev; ++k) {
    const MGLevel &F = P.lv[k], &C = P.lv[k + 1];
    mg_coarsen_kernel<<<mg_blocks(C.N), kThreads, 0, s>>>(
        mgeo(F), mgeo(C), m.ax + F.off, m.ay + F.off, m.az + F.off, m.diag + F.off, m.ax + C.off,
        m.ay + C.off, m.az + C.off, m.diag + C.off, m.dinv + C.off);
  }
  return hipGetLastError();
}

// z = V-cycle(r) for nrhs systems (skipping finished ones), partial sums of r.z;
// restrict0 false: the finest restriction has been done by the caller
hipError_t launch_mg_vcycle(const PGeom& g, const MGData& m, const double* r, double* z,
                            const CGState* st, int nrhs, hipStream_t s, bool restrict0) {
  const MGPlan& P = m.plan;
  const int L = P.nlev - 1, t = P.tail;
  const long long vs = P.vtotal;
  auto bvec = [&](int k) { return k == 0 ? r : m.b + P.lv[k].voff; };
  for (int k = restrict0 ? 0 : 1; k < t; ++k) {
    const MGLevel& C = P.lv[k + 1];
    mg_restrict_kernel<false><<<dim3(mg_blocks(8 * C.N), nrhs), kThreads, 0, s>>>(
        margs(m, k), mgeo(C), kMGOmega, bvec(k), k == 0 ? g.NP : vs, m.b + C.voff, vs, st,
        nullptr, nullptr, nullptr, nullptr, nullptr);
  }
  MGTailArgs T{};
  T.t = t;
  T.nt = L - t + 1;
  for (int k = t; k <= L; ++k) T.lv[k - t] = margs(m, k);
  for (int k = L + 1; k < t + kMGTailLevels; ++k) T.lv[k - t] = margs(m, L);   // unused slots
  mg_tail_kernel<<<dim3(1, nrhs), kMGTailNodes, 0, s>>>(T, kMGOmega, kMGCoarseSweeps,
                                                         m.b + P.lv[t].voff, m.u + P.lv[t].voff,
                                                         vs, st);
  for (int k = t - 1; k >= 1; --k) {
    const MGLevel &F = P.lv[k], &C = P.lv[k + 1];
    mg_correct_kernel<false><<<dim3(mg_blocks(F.N), nrhs), kThreads, 0, s>>>(
        margs(m, k), mgeo(C), kMGOmega, 1.0, m.b + F.voff, vs, m.u + C.voff, vs, m.u + F.voff,
        vs, nullptr, st);
  }
  const MGLevel& C1 = P.lv[1];
  mg_correct_kernel<true><<<dim3(sp_blocks(g.NP), nrhs), kThreads, 0, s>>>(
      margs(m, 0), mgeo(C1), kMGOmega, kMGAlpha, r, g.NP, m.u + C1.voff, vs, z, g.NP,
      m.partial_rz, st);
  return hipGetLastError();
}

hipError_t launch_mg_start(const PGeom& g, const MGData& m, const double* r, double* z,
                           CGState* st, int nrhs, hipStream_t s) {
  const hipError_t e = launch_mg_vcycle(g, m, r, z, st, nrhs, s, true);
  if (e != hipSuccess) return e;
  cg_rz_kernel<<<dim3(1, nrhs), kRedThreads, 0, s>>>(m.partial_rz, sp_blocks(g.NP), st);
  return hipGetLastError();
}

hipError_t launch_occupancy(int nev, const double* E, double n_holes, double kT, double* f,
                            double* mu, hipStream_t s) {
  if (nev < 1 || nev > 64) return hipErrorInvalidValue;
  occupancy_kernel<<<1, 64, 0, s>>>(nev, E, n_holes, kT, f, mu);
  return hipGetLastError();
}

hipError_t launch_rho(const PGeom& g, int ox, int oy, int oz, int nx, int ny, int nz, int nev,
                      const void* psi, long long vstride, const double* f, double inv_h3,
                      const double* rho_fixed, double* rho, double* density, hipStream_t s) {
  rho_kernel<<<sp_blocks(g.NP), kThreads, 0, s>>>((unsigned)g.NP, g.px, g.py, g.pz, 1.0 / g.py,
                                                  1.0 / g.pz, ox, oy, oz, nx, ny, nz, nev,
                                                  (const double2*)psi, vstride, f, inv_h3,
                                                  rho_fixed, rho, density);
  return hipGetLastError();
}

hipError_t launch_extract(int nx, int ny, int nz, const PGeom& g, int ox, int oy, int oz,
                          const double* V_off, const double* phi, double* V, hipStream_t s) {
  const long long NS = (long long)nx * ny * nz;
  extract_kernel<<<sp_blocks(NS), kThreads, 0, s>>>(NS, nx, ny, nz, g.py, g.pz, ox, oy, oz,
                                                    V_off, phi, V);
  return hipGetLastError();
}

hipError_t launch_residual_max(const PGeom& g, const double* phi_in, const double* phi_out,
                               double* F, double* partial, double* delta, hipStream_t s) {
  const int nb = sp_blocks(g.NP);
  residual_kernel<<<nb, kThreads, 0, s>>>(g.NP, phi_in, phi_out, F, partial);
  max_reduce_kernel<<<1, kThreads, 0, s>>>(partial, nb, delta);
  return hipGetLastError();
}

hipError_t launch_anderson(const PGeom& g, int k, int m, int slot, double mixing, double* x,
                           const double* F, double* histX, double* histF, double* G,
                           double* dots, double* gamma, double* partial, hipStream_t s) {
  if (k < 0 || k > 8 || k > m || m > 8) return hipErrorInvalidValue;
  const int nb = sp_blocks(g.NP);
  switch (k) {
    case 0: anderson_k<0>(g, nb, m, slot, mixing, x, F, histX, histF, G, dots, gamma, partial, s); break;
    case 1: anderson_k<1>(g, nb, m, slot, mixing, x, F, histX, histF, G, dots, gamma, partial, s); break;
    case 2: anderson_k<2>(g, nb, m, slot, mixing, x, F, histX, histF, G, dots, gamma, partial, s); break;
    case 3: anderson_k<3>(g, nb, m, slot, mixing, x, F, histX, histF, G, dots, gamma, partial, s); break;
    case 4: anderson_k<4>(g, nb, m, slot, mixing, x, F, histX, histF, G, dots, gamma, partial, s); break;
    case 5: anderson_k<5>(g, nb, m, slot, mixing, x, F, histX, histF, G, dots, gamma, partial, s); break;
    case 6: anderson_k<6>(g, nb, m, slot, mixing, x, F, histX, histF, G, dots, gamma, partial, s); break;
    case 7: anderson_k<7>(g, nb, m, slot, mixing, x, F, histX, histF, G, dots, gamma, partial, s); break;
    default: anderson_k<8>(g, nb, m, slot, mixing, x, F, histX, histF, G, dots, gamma, partial, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_pair_rhs(const PGeom& g, int ox, int oy, int oz, int nx, int ny, int nz, int M,
                           const void* phi, double h, double* rhs, hipStream_t s) {
  const int P = M * (M + 1) / 2;
  pair_rhs_kernel<<<dim3(sp_blocks(g.NP), P), kThreads, 0, s>>>(
      (unsigned)g.NP, g.px, g.py, g.pz, 1.0 / g.py, 1.0 / g.pz, ox, oy, oz, nx, ny, nz, M,
      static_cast<const double2*>(phi), 1.0 / (h * h * h), rhs);
  return hipGetLastError();
}

hipError_t launch_pair_potential_gather(const PGeom& g, int ox, int oy, int oz, int nx, int ny,
                                        int nz, int P, const double* V, double* Vc,
                                        hipStream_t s) {
  const long long NS = (long long)nx * ny * nz;
  pair_potential_gather_kernel<<<dim3((unsigned)((NS + kThreads - 1) / kThreads), P), kThreads, 0,
                                 s>>>(NS, nx, ny, nz, g.NP, g.py, g.pz, ox, oy, oz, V,
                                      reinterpret_cast<double2*>(Vc));
  return hipGetLastError();
}

hipError_t launch_pair_product(long long NS, int M, const void* phi, double* A, hipStream_t s) {
  pair_product_kernel<<<dim3((unsigned)((NS + kThreads - 1) / kThreads), M * M), kThreads, 0,
                        s>>>(NS, M, static_cast<const double2*>(phi),
                             reinterpret_cast<double2*>(A));
  return hipGetLastError();
}

hipError_t launch_ci_assemble(int M, const double* hsp, const double* Cs, double* H,
                              hipStream_t s) {
  const int n = 2 * M, K = n * (n - 1) / 2, P = M * (M + 1) / 2;
  ci_assemble_kernel<<<(K * K + kThreads - 1) / kThreads, kThreads, 0, s>>>(
      M, P, reinterpret_cast<const double2*>(hsp), reinterpret_cast<const double2*>(Cs),
      reinterpret_cast<double2*>(H));
  return hipGetLastError();
}

hipError_t launch_coulomb_expand(int M, const double* Cs, double* C, hipStream_t s) {
  const int P = M * (M + 1) / 2, n4 = M * M * M * M;
  coulomb_expand_kernel<<<(n4 + kThreads - 1) / kThreads, kThreads, 0, s>>>(
      M, P, reinterpret_cast<const double2*>(Cs), reinterpret_cast<double2*>(C));
  return hipGetLastError();
}

hipError_t launch_exchange(const double* E, double* J, hipStream_t s) {
  exchange_kernel<<<1, 64, 0, s>>>(E, J);
  return hipGetLastError();
}

}  // namespace hkp
