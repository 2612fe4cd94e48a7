// Matrix-free application of the finite-difference 6x6 hole Hamiltonian and
// the fused Chebyshev recurrence step
//
//     Y = alpha (H - shift) X + beta Y_old
//
// (the filter of the Rayleigh-Chebyshev subspace iteration, paper Sec. II.B).
//
// H in the |L S> basis (paper Eq. LK) is, per spin block, a 19-point stencil:
//   faces    -(E0/h^2) [ (L-M) S_ii + M (S_x + S_y + S_z) ]     on every component
//   edges    E0 N Ksym_ab coupling orbital components a <-> b (4 diagonal
//            neighbours in the (a,b) plane, two L-shaped Peierls paths averaged)
//   on-site  the orbital 3x3 block V + H_eps(r), the kinetic centre, spin-orbit
//            and Zeeman (a constant 6x6, evaluated in closed form)
// with L = g1+4g2, M = g1-2g2, N = 6 g3.
//
// Kernel design (gfx950): a workgroup owns a 64 x TY tile of (x, y) columns of
// one vector and marches along z.  Each plane (with a one-point halo ring) is
// staged through LDS once; every thread reads its 19-point neighbourhood from
// LDS and "pushes" the plane's contributions into three register accumulators
// for the output planes z-1, z and z+1.  The x-z and y-z edge couplings of a
// plane therefore need only that plane's x/y neighbours, so one plane of LDS
// per vector suffices.  Planes are double-buffered in LDS: the next plane is
// loaded into the other buffer while the current one is read (one barrier
// per plane), so HBM loads of one wave overlap the arithmetic of the others.  Output plane z-1
// is complete after plane z has been pushed and is written straight to HBM
// (alpha, beta and the old block fused in).  Workgroups are mapped to XCDs in
// contiguous runs so that the vectors of one tile share an L2.
#include <map>
#include <mutex>
#include <type_traits>

#include "hkp_internal.h"
#include "stencil_ops.h"

namespace hkp {

namespace {

using namespace sten;

template <typename T>
struct KArgs {
  const T* in;
  long long in_bstride;
  const void* old;
  long long old_bstride;
  void* out;
  long long out_bstride;
  const T* D;
  long long D_bstride;
  const T* wtab;
  const T* vtab;
  const double* coef;
  int coef_stride;
  double alpha, shift, beta;
  const int* active;
  const int* lock;
  const int* work;
  int batch;
  int zsplit, split_below;
  int nx, ny, nz, nvec;
  int tiles_x, tiles_y;
  int vgroup;   // vectors of one tile run side by side (1: vector-major)
  StencilConsts<T> k;
};

// DMA = true (tiles full along x): the 64 interior elements of every halo-tile
// row go global -> LDS directly (global_load_lds, no registers), issued one
// plane ahead and waited for at the end of the step; the two x-halo columns
// use ordinary loads.
// NC = 6: the full spinor (a wave per spin and row).  NC = 3: a spin-free orbital
// vector (X, Y, Z of one spin; no spin-orbit or field terms, so nothing couples
// it to the other spin): one wave per row and half the bytes.
// (FP32 steps without an old block are held to 128 VGPRs: four waves per SIMD)
template <typename T, typename TO, typename TW, int PH, bool STR, int TY, bool DMA, int NC = 6>
__global__ void __launch_bounds__(64 * TY * (NC / 3),
                                  (sizeof(T) == 4 && std::is_same<TO, void>::value && TY >= 2) ? 4 : 1)
stencil_kernel(KArgs<T> a) {
  static_assert(NC == 6 || (NC == 3 && PH == 0), "spin-free vectors carry no field terms");
  // LDS row: [pad] left halo, 64 interior, right halo [pad]; with FP32 DMA the
  // interior starts on a 16-byte boundary (column 2 of a 68-wide row)
  constexpr int C0 = (DMA && sizeof(T) == 4) ? 2 : 1;   // column of x = tx0
  constexpr int W = (DMA && sizeof(T) == 4) ? 68 : 66;
  constexpr int ROWS = TY + 2;
  constexpr int SLOTS = W * ROWS;
  constexpr int PLANE = SLOTS;        // elements per (buffer, component) plane
  constexpr int NT = 64 * TY * (NC / 3);   // (x, y, spin) threads
  constexpr int NS = (SLOTS + NT - 1) / NT;
  // double-buffered plane: [component][row][col] each (two distinct arrays, so the
  // compiler can tell the buffer being read from the one being filled)
  __shared__ cx<T> lds0[NC * PLANE];
  __shared__ cx<T> lds1[NC * PLANE];
  auto bufp = [&](auto BUF) -> cx<T>* {
    if constexpr (decltype(BUF)::value == 0) return lds0; else return lds1;
  };

  const int ntiles = a.tiles_x * a.tiles_y;
  // Workgroup order: groups of vgroup vectors; inside a group the vectors of
  // one tile are adjacent (they share the tile's on-site fields in L2) and the
  // tiles follow each other (neighbouring tiles march z side by side on one XCD,
  // so the halo rows they share hit in L2).  vgroup = 1 is vector-major order,
  // vgroup = nvec tile-major order.  With a work table the order runs over the
  // live (virtual) vectors of all members and the rest of the grid exits.
  // Launches with few live workgroups (locked vectors, converged members,
  // small grids) split every (vector, tile) into zs z-ranges so that more
  // workgroups share the chip; a range recomputes one plane on each side.
  // The grid holds zsplit x the unsplit count; the split is decided from the
  // live count, uniformly for the whole launch.
  int b, vec, tile, zs = 1, zc = 0;
  if (a.work) {
    const int nv = a.work[a.batch];
    const int nlw = nv * ntiles;
    if (a.zsplit > 1 && nlw < a.split_below && a.nz >= 8) zs = a.zsplit;
    const int nlive = nlw * zs;
    if ((int)blockIdx.x >= nlive) return;
    int logical = xcd_remap(blockIdx.x, nlive);
    zc = logical / nlw;   // z range outermost: one range of all tiles per XCD run
    logical -= zc * nlw;
    const int g = logical / (a.vgroup * ntiles);
    const int within = logical - g * a.vgroup * ntiles;
    const int gsize = min(a.vgroup, nv - g * a.vgroup);
    tile = within / gsize;
    const int u = g * a.vgroup + (within - tile * gsize);
    b = 0;
    while (a.work[b + 1] <= u) ++b;
    vec = (a.lock ? a.lock[b] : 0) + (u - a.work[b]);
  } else {
    const int nlw = (int)gridDim.x / a.zsplit;
    if (a.zsplit > 1 && nlw < a.split_below && a.nz >= 8) zs = a.zsplit;
    const int nlive = nlw * zs;
    if ((int)blockIdx.x >= nlive) return;
    int logical = xcd_remap(blockIdx.x, nlive);
    zc = logical / nlw;
    logical -= zc * nlw;
    const int per_b = ntiles * a.nvec;
    b = logical / per_b;
    const int r = logical - b * per_b;
    const int g = r / (a.vgroup * ntiles);
    const int within = r - g * a.vgroup * ntiles;
    const int gsize = min(a.vgroup, a.nvec - g * a.vgroup);
    tile = within / gsize;
    vec = g * a.vgroup + (within - tile * gsize);
    if (a.active && !a.active[b]) return;
    if (a.lock && vec < a.lock[b]) return;   // converged vectors are not filtered
  }
  const int tx0 = (tile % a.tiles_x) * 64;
  const int ty0 = (tile / a.tiles_x) * TY;

  const int nx = a.nx, ny = a.ny, nz = a.nz;
  // output planes [o0, o1) of this range; input planes p0..p1 feed them
  const int o0 = (zc * nz) / zs, o1 = ((zc + 1) * nz) / zs;
  const int p0 = o0 > 0 ? o0 - 1 : 0, p1 = o1 < nz ? o1 : nz - 1;
  const unsigned nxy = (unsigned)nx * (unsigned)ny;
  const unsigned N = nxy * (unsigned)nz;   // 6 N < 2^31 (checked on the host)
  const int lx = threadIdx.x, ly = threadIdx.y;
  // the spin is uniform across a wave (64 consecutive threads share threadIdx.z)
  const int sp = __builtin_amdgcn_readfirstlane(threadIdx.z);
  const int tid = lx + 64 * (ly + TY * sp);
  const int gx = tx0 + lx, gy = ty0 + ly;
  const bool mine = gx < nx && gy < ny;
  const int X = 3 * sp, F = 3 - X;      // own and flipped-spin component offsets

  T alpha, shift, beta;
  if (a.coef) {
    const double* c = a.coef + (long long)b * a.coef_stride;
    alpha = (T)c[0];
    shift = (T)c[1];
    beta = (T)c[2];
  } else {
    alpha = (T)a.alpha;
    shift = (T)a.shift;
    beta = (T)a.beta;
  }
  // TO = void: a launch without an old block (a step of the product-form filter,
  // or H X), compiled without its loads
  constexpr bool kOld = !std::is_same<TO, void>::value;
  using TOv = std::conditional_t<kOld, TO, T>;
  const bool has_old = kOld && a.old != nullptr && beta != (T)0;

  // uniform (scalar) bases; lane offsets are 32-bit element indices
  const T* __restrict__ in = a.in + 2 * ((long long)b * a.in_bstride + (long long)vec * NC * N);
  const TOv* __restrict__ oldp = has_old
      ? reinterpret_cast<const TOv*>(a.old) +
            2 * ((long long)b * a.old_bstride + (long long)vec * NC * N + (long long)X * N)
      : nullptr;
  TW* __restrict__ outp = reinterpret_cast<TW*>(a.out) +
                          2 * ((long long)b * a.out_bstride + (long long)vec * NC * N +
                               (long long)X * N);
  const T* __restrict__ D = a.D + (long long)b * a.D_bstride;
  const StencilConsts<T> k = a.k;
  // spin-dependent constants (sp is wave-uniform: scalar selects)
  const T dgs = sp == 0 ? k.dgU : k.dgD;
  const T ax = sp == 0 ? k.aUx : k.aDx, ay = sp == 0 ? k.aUy : k.aDy,
          az = sp == 0 ? k.aUz : k.aDz;
  const T sd3 = sp == 0 ? -k.d3 : k.d3;   // sign of the d3 f_Z and f_X spin-flip terms
  const T sby = sp == 0 ? -k.by : k.by;   // (bx -+ i by)

  // halo-tile slots this thread loads (clamped offset + mask; waves whose
  // slots are all inside the grid skip the mask)
  unsigned soff[NS];
  int sidx[NS];
  bool sval[NS], sin_[NS], wmask[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int slot = tid + s * NT;
    sin_[s] = slot < SLOTS;
    const int row = slot / W, colx = slot % W;
    const int x = tx0 + colx - C0, y = ty0 + row - 1;
    sval[s] = sin_[s] && x >= 0 && x < nx && y >= 0 && y < ny;
    soff[s] = sval[s] ? (unsigned)(y * nx + x) : 0u;
    sidx[s] = sin_[s] ? slot : 0;
    wmask[s] = !__all(sval[s] || !sin_[s]);
  }

  const unsigned col = mine ? (unsigned)(gy * nx + gx) : 0u;
  const int gxc = gx < nx ? gx : nx - 1;
  const int lb = (ly + 1) * W + (lx + C0);   // this thread's centre in an LDS plane

  cx<T> acc0[3], acc1[3], oldv[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) acc0[i] = acc1[i] = oldv[i] = mk<T>(0, 0);

  // next plane: loads issued before the current plane is computed, written to
  // the other LDS buffer after it (the wave's own arithmetic hides the latency)
  auto fetch = [&](int z, cx<T> (&v)[NS][NC]) {
    const unsigned zo = (unsigned)z * nxy;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (NS * NT > SLOTS && !sin_[s]) continue;
#pragma unroll
      for (int c = 0; c < NC; ++c) v[s][c] = ld(in + 2 * (size_t)((unsigned)c * N + zo + soff[s]));
    }
  };
  auto commit = [&](cx<T> (&v)[NS][NC], auto BUF) {
    cx<T>* dst = bufp(BUF);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (NS * NT > SLOTS && !sin_[s]) continue;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        cx<T> x = v[s][c];
        if (wmask[s] && !sval[s]) x = mk<T>(0, 0);
        dst[c * PLANE + sidx[s]] = x;
      }
    }
  };

  // ---- DMA staging: row loads spread over the workgroup's waves
  constexpr int NW = TY * (NC / 3);
  const int wave = __builtin_amdgcn_readfirstlane(ly + TY * sp);
  auto dma_plane = [&](int z, auto BUF) {
    cx<T>* dst = bufp(BUF);
    const unsigned zo = (unsigned)z * nxy;
    for (int j = wave; j < NC * ROWS; j += NW) {
      const int c = j / ROWS, r = j % ROWS;
      const int y = ty0 + r - 1;
      if (y < 0 || y >= ny) continue;
      const T* src = in + 2 * (size_t)((unsigned)c * N + zo + (unsigned)(y * nx + tx0)) +
                     (sizeof(T) == 8 ? 2 : 4) * lx;
      cx<T>* drow = dst + c * PLANE + r * W + C0;
      if (sizeof(T) == 8 || lx < 32)
        dma16(src, drow);
    }
  };
  // x-halo columns: element e of 12 ROWS per plane (side, component, row)
  const int he = tid;
  const bool hown = he < 2 * NC * ROWS;
  const int hside = he & 1, hc = (he >> 1) % NC, hr = (he >> 1) / NC;
  const int hx = hside ? tx0 + 64 : tx0 - 1, hy = ty0 + hr - 1;
  const bool hval = hown && hx >= 0 && hx < nx && hy >= 0 && hy < ny;
  const unsigned hoff = hval ? (unsigned)(hc * N + hy * nx + hx) : 0u;
  const int hidx = hc * PLANE + hr * W + (hside ? C0 + 64 : C0 - 1);
  auto halo_load = [&](int z) -> cx<T> {
    cx<T> v = mk<T>(0, 0);
    if (hval) v = ld(in + 2 * (size_t)(hoff + (unsigned)z * nxy));
    return v;
  };
  auto halo_commit = [&](cx<T> v, auto BUF) {
    if (hown) bufp(BUF)[hidx] = v;
  };

  auto load_old = [&](int z) {
    if (!kOld || !has_old || !mine) return;
    const unsigned o = (unsigned)z * nxy + col;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cx<TOv> q = ld_stream(oldp + 2 * (size_t)((unsigned)i * N + o));
      oldv[i] = mk<T>((T)q.r, (T)q.i);
    }
  };
  auto finalize = [&](int z) {
    if (!mine) return;
    const unsigned o = (unsigned)z * nxy + col;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cx<T> r = scl(alpha, acc0[i]);
      if (kOld && has_old) r = fma_s(r, beta, oldv[i]);
      stg_stream<TW>(outp, (long long)((unsigned)i * N + o), r);
    }
  };

  // link phases (GPU gauge) as a rolling window over planes z-1, z, z+1,
  // loaded one plane ahead: x-links per plane (w), y-links per (plane, column)
  // (v; with Bz = 0, PH == 1, uniform over the plane); PH == 2 also needs the
  // y-links of the neighbouring columns in plane z (vx+, vx-)
  const int xc = PH == 2 ? gxc : 0;
  const int xcp = gxc + 1 < nx ? gxc + 1 : gxc, xcm = gxc > 0 ? gxc - 1 : 0;
  cx<T> pw[3], pv[3], pvxp, pvxm;
  if constexpr (PH != 0) {
    const int zm = p0 > 0 ? p0 - 1 : 0, z1 = p0 + 1 < nz ? p0 + 1 : nz - 1;
    pw[0] = ld(a.wtab + 2 * zm);
    pw[1] = ld(a.wtab + 2 * p0);
    pw[2] = ld(a.wtab + 2 * z1);
    pv[0] = ld(a.vtab + 2 * (zm * nx + xc));
    pv[1] = ld(a.vtab + 2 * (p0 * nx + xc));
    pv[2] = ld(a.vtab + 2 * (z1 * nx + xc));
    if constexpr (PH == 2) {
      pvxp = ld(a.vtab + 2 * (p0 * nx + xcp));
      pvxm = ld(a.vtab + 2 * (p0 * nx + xcm));
    }
  }

  // on-site fields of this column, loaded one plane ahead (d00 d11 d22 d12 d02 d01;
  // without strain only the first)
  constexpr int ND = STR ? 6 : 1;
  auto load_d = [&](int z, T (&d)[ND]) {
    const unsigned pz = (unsigned)z * nxy + col;
#pragma unroll
    for (int i = 0; i < ND; ++i) d[i] = D[(unsigned)i * N + pz];
  };
  T cd[ND];
  load_d(p0, cd);

  auto step = [&](int z, auto BUF) {
    constexpr int cur = decltype(BUF)::value;
    // loads in the order they are needed (the memory counter retires them in
    // order): next plane's phases, this plane's on-site fields, the old block
    // for the output plane, the next plane's halo, the next plane's rows
    cx<T> nw, nv, nvxp, nvxm;
    if constexpr (PH != 0) {
      const int z2 = z + 2 < nz ? z + 2 : nz - 1, z1 = z + 1 < nz ? z + 1 : nz - 1;
      nw = ld(a.wtab + 2 * z2);
      nv = ld(a.vtab + 2 * (z2 * nx + xc));
      if constexpr (PH == 2) {
        nvxp = ld(a.vtab + 2 * (z1 * nx + xcp));
        nvxm = ld(a.vtab + 2 * (z1 * nx + xcm));
      }
    }
    // the next plane goes to the other buffer while this one is read; the
    // barrier at the end of the step publishes it and retires this buffer
    // FP32: loads of the next plane issued before the arithmetic and written to
    // LDS after it (latency hidden by this wave's own work); FP64 writes them
    // at once (its register budget is already exhausted by the arithmetic)
    constexpr bool late = sizeof(T) == 4;
    T nd[ND];
    load_d(z + 1 < nz ? z + 1 : z, nd);
    if (z - 1 >= o0) load_old(z - 1);
    cx<T> nxt[DMA ? 1 : NS][NC];
    cx<T> hv = mk<T>(0, 0);
    const bool more = z + 1 <= p1;
    if constexpr (!DMA) {
      if (more) {
        fetch(z + 1, nxt);
        if constexpr (!late) commit(nxt, IC<1 - cur>{});
      }
    } else {
      if (more) {
        hv = halo_load(z + 1);
        dma_plane(z + 1, IC<1 - cur>{});
      }
    }
    // (indices stay inside cd for ND = 1; the strain terms are then zero)
    const T d00 = cd[0], d11 = cd[STR ? 1 : 0], d22 = cd[STR ? 2 : 0];
    const T d12 = STR ? cd[STR ? 3 : 0] : (T)0;
    const T d02 = STR ? cd[STR ? 4 : 0] : (T)0;
    const T d01 = STR ? cd[STR ? 5 : 0] : (T)0;
    const cx<T>* L = bufp(IC<cur>{}) + lb;
    cx<T> acc2[3];
    push_plane<T, PH, STR, NC, PLANE, W>(L, X, F, k, dgs, ax, ay, az, sd3, sby, shift, pw, pv,
                                         pvxp, pvxm, d00, d11, d22, d12, d02, d01, acc0, acc1,
                                         acc2);

    // the output plane's stores (and the wait for the old block, which the
    // compiler extends to every load in flight, the next plane's copy included)
    // after all of this plane's arithmetic
    settle(acc1);
    settle(acc2);
    if (z - 1 >= o0) finalize(z - 1);
    if constexpr (DMA) {
      if (more) halo_commit(hv, IC<1 - cur>{});
    } else if constexpr (late) {
      if (more) commit(nxt, IC<1 - cur>{});
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      acc0[i] = acc1[i];
      acc1[i] = acc2[i];
    }
#pragma unroll
    for (int i = 0; i < ND; ++i) cd[i] = nd[i];
    if constexpr (PH != 0) {
      pw[0] = pw[1];
      pw[1] = pw[2];
      pw[2] = nw;
      pv[0] = pv[1];
      pv[1] = pv[2];
      pv[2] = nv;
      if constexpr (PH == 2) {
        pvxp = nvxp;
        pvxm = nvxm;
      }
    }
    __syncthreads();
  };

  if constexpr (DMA) {
    // rows outside the grid are never loaded: zero both buffers once
    for (int i = tid; i < NC * PLANE; i += NT) {
      lds0[i] = mk<T>(0, 0);
      lds1[i] = mk<T>(0, 0);
    }
    __syncthreads();
    halo_commit(halo_load(p0), IC<0>{});
    dma_plane(p0, IC<0>{});
  } else {
    cx<T> first[NS][NC];
    fetch(p0, first);
    commit(first, IC<0>{});
  }
  __syncthreads();
  for (int z = p0; z <= p1; z += 2) {
    step(z, IC<0>{});
    if (z + 1 <= p1) step(z + 1, IC<1>{});
  }
  if (o1 == nz) {   // the last plane has no successor to complete it
    load_old(nz - 1);
    finalize(nz - 1);
  }
}

// workgroups of this kernel resident on the whole device at once (occupancy
// query, cached per kernel)
template <typename K>
int resident_workgroups(K kernel, int threads) {
  static std::mutex mu;
  static std::map<const void*, int> cache;
  const void* key = reinterpret_cast<const void*>(kernel);
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;   // unknown: never split
  }
  const int r = per_cu * cus;
  cache[key] = r;
  return r;
}

template <typename T, typename TO, typename TW, int PH, bool STR, int NC = 6>
hipError_t launch_t(const StencilLaunch& L, const StencilConsts<double>& c, hipStream_t s) {
  KArgs<T> a;
  a.in = reinterpret_cast<const T*>(L.in);
  a.in_bstride = L.in_bstride;
  a.old = L.old;
  a.old_bstride = L.old_bstride;
  a.out = L.out;
  a.out_bstride = L.out_bstride;
  a.D = reinterpret_cast<const T*>(L.D);
  a.D_bstride = L.D_bstride;
  a.wtab = reinterpret_cast<const T*>(L.wtab);
  a.vtab = reinterpret_cast<const T*>(L.vtab);
  a.coef = L.coef.coef;
  a.coef_stride = L.coef.stride;
  a.alpha = L.coef.alpha;
  a.shift = L.coef.shift;
  a.beta = L.coef.beta;
  a.active = L.active;
  a.lock = L.lock;
  a.work = L.work;
  a.batch = L.batch;
  a.nx = L.nx;
  a.ny = L.ny;
  a.nz = L.nz;
  a.nvec = L.nvec;
  a.vgroup = L.vgroup < 1 ? 1 : (L.vgroup > L.nvec ? L.nvec : L.vgroup);
  a.k = cast_consts<T>(c);
  const int ty = L.tile_y;
  a.tiles_x = (L.nx + 63) / 64;
  a.tiles_y = (L.ny + ty - 1) / ty;
  const long long nwg = (long long)a.tiles_x * a.tiles_y * L.nvec * L.batch;
  if (nwg <= 0) return hipSuccess;
  // z split: 0 never, 1 when fewer live workgroups than three resident waves,
  // 2 always (tests)
  a.zsplit = L.zsplit > 0 ? 2 : 1;
  if (nwg * a.zsplit > 0x7fffffffLL) return hipErrorInvalidValue;
  dim3 grid((unsigned)(nwg * a.zsplit));
  auto go = [&](auto kernel, dim3 block) {
    a.split_below = L.zsplit >= 2 ? 0x7fffffff
                  : (L.zsplit == 1 ? 3 * resident_workgroups(kernel, (int)(block.x * block.y * block.z)) : 0);
    kernel<<<grid, block, 0, s>>>(a);
  };
  constexpr unsigned NSP = NC / 3;   // spin waves per row
  if (L.dma && L.nx % 64 == 0) {
    switch (ty) {
      case 1: go(stencil_kernel<T, TO, TW, PH, STR, 1, true, NC>, dim3(64, 1, NSP)); break;
      case 2: go(stencil_kernel<T, TO, TW, PH, STR, 2, true, NC>, dim3(64, 2, NSP)); break;
      case 4: go(stencil_kernel<T, TO, TW, PH, STR, 4, true, NC>, dim3(64, 4, NSP)); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (ty) {
    case 1: go(stencil_kernel<T, TO, TW, PH, STR, 1, false, NC>, dim3(64, 1, NSP)); break;
    case 2: go(stencil_kernel<T, TO, TW, PH, STR, 2, false, NC>, dim3(64, 2, NSP)); break;
    case 4: go(stencil_kernel<T, TO, TW, PH, STR, 4, false, NC>, dim3(64, 4, NSP)); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, typename TO, typename TW>
hipError_t launch_ph(const StencilLaunch& L, const StencilConsts<double>& c, hipStream_t s) {
  // 0: no field; 1: Bz = 0 (all link phases uniform over a z-plane); 2: general
  const int ph = L.wtab == nullptr ? 0 : (L.phase_general ? 2 : 1);
  if (L.ncomp == 3) {   // spin-free orbital vectors: zero field only
    if (ph != 0) return hipErrorInvalidValue;
    return L.strain ? launch_t<T, TO, TW, 0, true, 3>(L, c, s)
                    : launch_t<T, TO, TW, 0, false, 3>(L, c, s);
  }
  if (ph == 2)
    return L.strain ? launch_t<T, TO, TW, 2, true>(L, c, s) : launch_t<T, TO, TW, 2, false>(L, c, s);
  if (ph == 1)
    return L.strain ? launch_t<T, TO, TW, 1, true>(L, c, s) : launch_t<T, TO, TW, 1, false>(L, c, s);
  return L.strain ? launch_t<T, TO, TW, 0, true>(L, c, s) : launch_t<T, TO, TW, 0, false>(L, c, s);
}

}  // namespace

StencilConsts<double> make_consts(const hkp_material& m, double h, const double B[3]) {
  const double L = m.gamma1 + 4.0 * m.gamma2, M = m.gamma1 - 2.0 * m.gamma2;
  const double Nn = 6.0 * m.gamma3;
  const double eh = kE0 / (h * h);
  StencilConsts<double> c;
  c.cLM = -eh * (L - M);
  c.cM = -eh * M;
  c.czZ = -eh * L;
  c.cN8 = -kE0 * Nn / (8.0 * h * h);
  const double k0 = 2.0 * eh * (L + 2.0 * M);
  const double d3 = m.delta_so_eV / 3.0;
  const double zb = kMuB * B[2];
  c.dgU = k0 + d3 + zb;
  c.dgD = k0 + d3 - zb;
  const double g = kMuB * (3.0 * m.kappa - 1.0);
  c.aUx = g * B[0];
  c.aUy = g * B[1];
  c.aUz = g * B[2] - d3;
  c.aDx = g * B[0];
  c.aDy = g * B[1];
  c.aDz = g * B[2] + d3;
  c.d3 = d3;
  c.bx = kMuB * B[0];
  c.by = kMuB * B[1];
  return c;
}

template <typename T>
StencilConsts<T> cast_consts(const StencilConsts<double>& c) {
  StencilConsts<T> o;
  o.cLM = (T)c.cLM; o.cM = (T)c.cM; o.czZ = (T)c.czZ; o.cN8 = (T)c.cN8;
  o.dgU = (T)c.dgU; o.dgD = (T)c.dgD;
  o.aUx = (T)c.aUx; o.aUy = (T)c.aUy; o.aUz = (T)c.aUz;
  o.aDx = (T)c.aDx; o.aDy = (T)c.aDy; o.aDz = (T)c.aDz;
  o.d3 = (T)c.d3; o.bx = (T)c.bx; o.by = (T)c.by;
  return o;
}
template StencilConsts<double> cast_consts<double>(const StencilConsts<double>&);
template StencilConsts<float> cast_consts<float>(const StencilConsts<double>&);

hipError_t launch_stencil(const StencilLaunch& L, const StencilConsts<double>& c,
                          hipStream_t s) {
  if (L.fp64) {
    if (!L.out_fp64) return hipErrorInvalidValue;
    return L.old ? launch_ph<double, double, double>(L, c, s)
                 : launch_ph<double, void, double>(L, c, s);
  }
  if (!L.old)   // no old block: H X, or a step of the product-form filter
    return L.out_fp64 ? launch_ph<float, void, double>(L, c, s)
                      : launch_ph<float, void, float>(L, c, s);
  // FP32 stencil: old may be FP64 (the first recurrence step reads X) and the
  // output FP64 (the last step feeds the FP64 orthonormalisation)
  if (L.old_fp64) {
    return L.out_fp64 ? launch_ph<float, double, double>(L, c, s)
                      : launch_ph<float, double, float>(L, c, s);
  }
  return L.out_fp64 ? launch_ph<float, float, double>(L, c, s)
                    : launch_ph<float, float, float>(L, c, s);
}

}  // namespace hkp
