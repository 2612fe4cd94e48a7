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
// per vector suffices.  The next plane is prefetched into registers while the
// current one is computed, so HBM loads overlap arithmetic.  Output plane z-1
// is complete after plane z has been pushed and is written straight to HBM
// (alpha, beta and the old block fused in).  Workgroups are mapped to XCDs in
// contiguous runs so that the vectors of one tile share an L2.
#include "hkp_internal.h"

namespace hkp {

namespace {

template <typename T> struct V2;
template <> struct V2<double> { using type = double2; };
template <> struct V2<float> { using type = float2; };

template <typename T>
struct cx {
  T r, i;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T>
__device__ __forceinline__ cx<T> add(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <typename T>
__device__ __forceinline__ cx<T> sub(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <typename T>
__device__ __forceinline__ cx<T> scl(T s, cx<T> a) { return {s * a.r, s * a.i}; }
// a + s * b
template <typename T>
__device__ __forceinline__ cx<T> fma_s(cx<T> a, T s, cx<T> b) {
  return {fma(s, b.r, a.r), fma(s, b.i, a.i)};
}
template <typename T>
__device__ __forceinline__ cx<T> mul(cx<T> a, cx<T> b) {
  return {fma(a.r, b.r, -a.i * b.i), fma(a.r, b.i, a.i * b.r)};
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.r, -a.i}; }
// i * a
template <typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.i, a.r}; }
// w a - conj(w) b
template <typename T>
__device__ __forceinline__ cx<T> wdiff(cx<T> w, cx<T> a, cx<T> b) {
  // w a - conj(w) b = wr (a - b) + i wi (a + b)
  cx<T> d = sub(a, b), s = add(a, b);
  return {fma(w.r, d.r, -w.i * s.i), fma(w.r, d.i, w.i * s.r)};
}
// w a + conj(w) b
template <typename T>
__device__ __forceinline__ cx<T> wsum(cx<T> w, cx<T> a, cx<T> b) {
  cx<T> d = sub(a, b), s = add(a, b);
  return {fma(w.r, s.r, -w.i * d.i), fma(w.r, s.i, w.i * d.r)};
}

template <typename T>
__device__ __forceinline__ cx<T> ld(const T* p) {
  typename V2<T>::type v = *reinterpret_cast<const typename V2<T>::type*>(p);
  return {v.x, v.y};
}
template <typename T>
__device__ __forceinline__ cx<T> ldg(const void* base, long long idx) {
  return ld(reinterpret_cast<const T*>(base) + 2 * idx);
}

template <typename TW, typename T>
__device__ __forceinline__ void stg(void* base, long long idx, cx<T> v) {
  typename V2<TW>::type o;
  o.x = static_cast<TW>(v.r);
  o.y = static_cast<TW>(v.i);
  reinterpret_cast<typename V2<TW>::type*>(base)[idx] = o;
}

__device__ __forceinline__ int xcd_remap(int wg, int nwg) {
  // hardware places workgroup wg on XCD wg % 8; give every XCD a contiguous
  // run of logical workgroups
  const int x = wg & 7, idx = wg >> 3;
  const int per = nwg >> 3, rem = nwg & 7;
  return x * per + (x < rem ? x : rem) + idx;
}

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
  int nx, ny, nz, nvec;
  int tiles_x, tiles_y;
  StencilConsts<T> k;
};

template <typename T, typename TO, typename TW, bool PH, bool STR, int TY>
__global__ void __launch_bounds__(64 * TY)
stencil_kernel(KArgs<T> a) {
  constexpr int W = 66;               // 64 + halo
  constexpr int ROWS = TY + 2;
  constexpr int SLOTS = W * ROWS;
  constexpr int NT = 64 * TY;
  constexpr int NS = (SLOTS + NT - 1) / NT;
  __shared__ cx<T> lds[6][ROWS][W];

  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int vec = logical % a.nvec;
  int rest = logical / a.nvec;
  const int tile = rest % (a.tiles_x * a.tiles_y);
  const int b = rest / (a.tiles_x * a.tiles_y);
  if (a.active && !a.active[b]) return;
  const int tx0 = (tile % a.tiles_x) * 64;
  const int ty0 = (tile / a.tiles_x) * TY;

  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const long long nxy = (long long)nx * ny;
  const long long N = nxy * nz;
  const int tid = threadIdx.x + 64 * threadIdx.y;
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int gx = tx0 + lx, gy = ty0 + ly;
  const bool mine = gx < nx && gy < ny;

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
  const bool has_old = a.old != nullptr && beta != (T)0;

  const T* in = a.in + 2 * ((long long)b * a.in_bstride + (long long)vec * 6 * N);
  const long long old_off = (long long)b * a.old_bstride + (long long)vec * 6 * N;
  const long long out_off = (long long)b * a.out_bstride + (long long)vec * 6 * N;
  const T* D = a.D + (long long)b * a.D_bstride;
  const StencilConsts<T> k = a.k;

  // slot -> (row, col) of the halo tile owned by this thread for loads
  int srow[NS], scol[NS];
  bool sval[NS];
  long long soff[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int slot = tid + s * NT;
    srow[s] = slot / W;
    scol[s] = slot % W;
    const int x = tx0 + scol[s] - 1, y = ty0 + srow[s] - 1;
    sval[s] = slot < SLOTS && x >= 0 && x < nx && y >= 0 && y < ny;
    soff[s] = sval[s] ? (long long)y * nx + x : 0;
  }

  cx<T> pf[NS][6];
  auto prefetch = [&](int z) {
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int c = 0; c < 6; ++c)
        pf[s][c] = sval[s] ? ld(in + 2 * ((long long)c * N + (long long)z * nxy + soff[s]))
                           : mk<T>(0, 0);
  };

  cx<T> acc0[6], acc1[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) acc0[c] = acc1[c] = mk<T>(0, 0);

  const long long col = mine ? (long long)gy * nx + gx : 0;
  const int gxc = gx < nx ? gx : nx - 1;

  auto finalize = [&](int z, cx<T>* acc) {
    if (!mine) return;
    const long long base = (long long)z * nxy + col;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      cx<T> r = scl(alpha, acc[c]);
      if (has_old) {
        cx<TO> o = ldg<TO>(a.old, old_off + (long long)c * N + base);
        r = fma_s(r, beta, mk<T>((T)o.r, (T)o.i));
      }
      stg<TW>(a.out, out_off + (long long)c * N + base, r);
    }
  };

  prefetch(0);
  for (int z = 0; z < nz; ++z) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (tid + s * NT < SLOTS)
#pragma unroll
        for (int c = 0; c < 6; ++c) lds[c][srow[s]][scol[s]] = pf[s][c];
    __syncthreads();
    if (z + 1 < nz) prefetch(z + 1);

    // ---- neighbourhood of (gx, gy, z) from LDS
    const int r0 = ly + 1, c0 = lx + 1;
    cx<T> own[6], xp[6], xm[6], yp[6], ym[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      own[c] = lds[c][r0][c0];
      xp[c] = lds[c][r0][c0 + 1];
      xm[c] = lds[c][r0][c0 - 1];
      yp[c] = lds[c][r0 + 1][c0];
      ym[c] = lds[c][r0 - 1][c0];
    }

    // ---- phases (GPU gauge): x-links per plane, y-links per (plane, column)
    cx<T> w0, wm, wp, v0, vm, vp, vxp, vxm;
    if constexpr (PH) {
      const int zm = z > 0 ? z - 1 : 0, zq = z + 1 < nz ? z + 1 : nz - 1;
      w0 = ld(a.wtab + 2 * z);
      wm = ld(a.wtab + 2 * zm);
      wp = ld(a.wtab + 2 * zq);
      v0 = ld(a.vtab + 2 * ((long long)z * nx + gxc));
      vm = ld(a.vtab + 2 * ((long long)zm * nx + gxc));
      vp = ld(a.vtab + 2 * ((long long)zq * nx + gxc));
      vxp = ld(a.vtab + 2 * ((long long)z * nx + (gxc + 1 < nx ? gxc + 1 : gxc)));
      vxm = ld(a.vtab + 2 * ((long long)z * nx + (gxc > 0 ? gxc - 1 : 0)));
    }

    cx<T> acc2[6];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int X = 3 * s, Y = 3 * s + 1, Z = 3 * s + 2;
      // faces in the plane
      cx<T> Sx[3], Sy[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        if constexpr (PH) {
          Sx[i] = wsum(w0, xp[X + i], xm[X + i]);
          Sy[i] = wsum(v0, yp[X + i], ym[X + i]);
        } else {
          Sx[i] = add(xp[X + i], xm[X + i]);
          Sy[i] = add(yp[X + i], ym[X + i]);
        }
      }
      acc1[X] = fma_s(acc1[X], k.cLM, Sx[0]);
      acc1[Y] = fma_s(acc1[Y], k.cLM, Sy[1]);
#pragma unroll
      for (int i = 0; i < 3; ++i) acc1[X + i] = fma_s(acc1[X + i], k.cM, add(Sx[i], Sy[i]));

      // x-y edges (in plane): couple X <-> Y
      {
        const cx<T> fY_pp = lds[Y][r0 + 1][c0 + 1], fY_pm = lds[Y][r0 - 1][c0 + 1];
        const cx<T> fY_mp = lds[Y][r0 + 1][c0 - 1], fY_mm = lds[Y][r0 - 1][c0 - 1];
        const cx<T> fX_pp = lds[X][r0 + 1][c0 + 1], fX_pm = lds[X][r0 - 1][c0 + 1];
        const cx<T> fX_mp = lds[X][r0 + 1][c0 - 1], fX_mm = lds[X][r0 - 1][c0 - 1];
        if constexpr (PH) {
          // P(sx, sy) = w^sx [ v(x+sx)^sy + v(x)^sy ]
          const cx<T> ppp = mul(w0, add(vxp, v0));
          const cx<T> ppm = mul(w0, conj(add(vxp, v0)));
          const cx<T> pmp = mul(conj(w0), add(vxm, v0));
          const cx<T> pmm = mul(conj(w0), conj(add(vxm, v0)));
          cx<T> eY = sub(add(mul(ppp, fY_pp), mul(pmm, fY_mm)), add(mul(ppm, fY_pm), mul(pmp, fY_mp)));
          cx<T> eX = sub(add(mul(ppp, fX_pp), mul(pmm, fX_mm)), add(mul(ppm, fX_pm), mul(pmp, fX_mp)));
          acc1[X] = fma_s(acc1[X], k.cN8, eY);
          acc1[Y] = fma_s(acc1[Y], k.cN8, eX);
        } else {
          cx<T> eY = sub(add(fY_pp, fY_mm), add(fY_pm, fY_mp));
          cx<T> eX = sub(add(fX_pp, fX_mm), add(fX_pm, fX_mp));
          const T c2 = k.cN8 + k.cN8;
          acc1[X] = fma_s(acc1[X], c2, eY);
          acc1[Y] = fma_s(acc1[Y], c2, eX);
        }
      }

      // z faces: pushed to z-1 and z+1
      acc0[X] = fma_s(acc0[X], k.cM, own[X]);
      acc0[Y] = fma_s(acc0[Y], k.cM, own[Y]);
      acc0[Z] = fma_s(acc0[Z], k.czZ, own[Z]);
      acc2[X] = scl(k.cM, own[X]);
      acc2[Y] = scl(k.cM, own[Y]);
      acc2[Z] = scl(k.czZ, own[Z]);

      // x-z and y-z edges of this plane, pushed to z-1 (sz = +1) and z+1 (sz = -1)
      if constexpr (PH) {
        const cx<T> wu = add(wm, w0), wd = add(wp, w0);   // path averages (x2)
        const cx<T> vu = add(vm, v0), vd = add(vp, v0);
        acc0[X] = fma_s(acc0[X], k.cN8, wdiff(wu, xp[Z], xm[Z]));
        acc0[Z] = fma_s(acc0[Z], k.cN8, wdiff(wu, xp[X], xm[X]));
        acc0[Y] = fma_s(acc0[Y], k.cN8, wdiff(vu, yp[Z], ym[Z]));
        acc0[Z] = fma_s(acc0[Z], k.cN8, wdiff(vu, yp[Y], ym[Y]));
        acc2[X] = fma_s(acc2[X], -k.cN8, wdiff(wd, xp[Z], xm[Z]));
        acc2[Z] = fma_s(acc2[Z], -k.cN8, wdiff(wd, xp[X], xm[X]));
        acc2[Y] = fma_s(acc2[Y], -k.cN8, wdiff(vd, yp[Z], ym[Z]));
        acc2[Z] = fma_s(acc2[Z], -k.cN8, wdiff(vd, yp[Y], ym[Y]));
      } else {
        const T c2 = k.cN8 + k.cN8;
        const cx<T> dxZ = sub(xp[Z], xm[Z]), dxX = sub(xp[X], xm[X]);
        const cx<T> dyZ = sub(yp[Z], ym[Z]), dyY = sub(yp[Y], ym[Y]);
        acc0[X] = fma_s(acc0[X], c2, dxZ);
        acc0[Z] = fma_s(acc0[Z], c2, add(dxX, dyY));
        acc0[Y] = fma_s(acc0[Y], c2, dyZ);
        acc2[X] = fma_s(acc2[X], -c2, dxZ);
        acc2[Z] = fma_s(acc2[Z], -c2, add(dxX, dyY));
        acc2[Y] = fma_s(acc2[Y], -c2, dyZ);
      }
    }

    // ---- on-site: orbital block (V + strain) on both spins, constants, SO/Zeeman
    {
      const long long p = (long long)z * nxy + col;
      T d00, d11, d22, d12 = 0, d02 = 0, d01 = 0;
      if constexpr (STR) {
        d00 = D[p];
        d11 = D[N + p];
        d22 = D[2 * N + p];
        d12 = D[3 * N + p];
        d02 = D[4 * N + p];
        d01 = D[5 * N + p];
      } else {
        d00 = d11 = d22 = D[p];
      }
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int X = 3 * s;
        const T dg = (s == 0 ? k.dgU : k.dgD) - shift;
        const cx<T> u0 = own[X], u1 = own[X + 1], u2 = own[X + 2];
        cx<T> r0v = scl(d00 + dg, u0), r1v = scl(d11 + dg, u1), r2v = scl(d22 + dg, u2);
        if constexpr (STR) {
          r0v = fma_s(fma_s(r0v, d01, u1), d02, u2);
          r1v = fma_s(fma_s(r1v, d01, u0), d12, u2);
          r2v = fma_s(fma_s(r2v, d02, u0), d12, u1);
        }
        // i (a x u)
        const T ax = s == 0 ? k.aUx : k.aDx, ay = s == 0 ? k.aUy : k.aDy,
                az = s == 0 ? k.aUz : k.aDz;
        cx<T> c0v, c1v, c2v;
        if constexpr (PH) {
          c0v = sub(scl(ay, u2), scl(az, u1));
          c1v = sub(scl(az, u0), scl(ax, u2));
          c2v = sub(scl(ax, u1), scl(ay, u0));
        } else {
          c0v = scl(-az, u1);
          c1v = scl(az, u0);
          c2v = mk<T>(0, 0);
        }
        r0v = add(r0v, mul_i(c0v));
        r1v = add(r1v, mul_i(c1v));
        r2v = add(r2v, mul_i(c2v));
        // spin flip: up <- -d3 (v_Z, -i v_Z, -v_X + i v_Y) + (bx - i by) v   (v = down)
        //            dn <- -d3 (-v_Z, -i v_Z, v_X + i v_Y) + (bx + i by) v   (v = up)
        const int F = 3 - X;
        const cx<T> f0 = own[F], f1 = own[F + 1], f2 = own[F + 2];
        if (s == 0) {
          r0v = fma_s(r0v, -k.d3, f2);
          r1v = fma_s(r1v, k.d3, mul_i(f2));
          r2v = fma_s(r2v, -k.d3, sub(mul_i(f1), f0));
        } else {
          r0v = fma_s(r0v, k.d3, f2);
          r1v = fma_s(r1v, k.d3, mul_i(f2));
          r2v = fma_s(r2v, -k.d3, add(mul_i(f1), f0));
        }
        if constexpr (PH) {
          const cx<T> bz = mk<T>(k.bx, s == 0 ? -k.by : k.by);
          r0v = add(r0v, mul(bz, f0));
          r1v = add(r1v, mul(bz, f1));
          r2v = add(r2v, mul(bz, f2));
        }
        acc1[X] = add(acc1[X], r0v);
        acc1[X + 1] = add(acc1[X + 1], r1v);
        acc1[X + 2] = add(acc1[X + 2], r2v);
      }
    }

    if (z >= 1) finalize(z - 1, acc0);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      acc0[c] = acc1[c];
      acc1[c] = acc2[c];
    }
  }
  finalize(nz - 1, acc0);
}

template <typename T, typename TO, typename TW, bool PH, bool STR>
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
  a.nx = L.nx;
  a.ny = L.ny;
  a.nz = L.nz;
  a.nvec = L.nvec;
  a.k = cast_consts<T>(c);
  const int ty = L.tile_y;
  a.tiles_x = (L.nx + 63) / 64;
  a.tiles_y = (L.ny + ty - 1) / ty;
  const long long nwg = (long long)a.tiles_x * a.tiles_y * L.nvec * L.batch;
  if (nwg <= 0) return hipSuccess;
  if (nwg > 0x7fffffffLL) return hipErrorInvalidValue;
  dim3 grid((unsigned)nwg);
  switch (ty) {
    case 1: stencil_kernel<T, TO, TW, PH, STR, 1><<<grid, dim3(64, 1), 0, s>>>(a); break;
    case 2: stencil_kernel<T, TO, TW, PH, STR, 2><<<grid, dim3(64, 2), 0, s>>>(a); break;
    case 4: stencil_kernel<T, TO, TW, PH, STR, 4><<<grid, dim3(64, 4), 0, s>>>(a); break;
    case 8: stencil_kernel<T, TO, TW, PH, STR, 8><<<grid, dim3(64, 8), 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, typename TO, typename TW>
hipError_t launch_ph(const StencilLaunch& L, const StencilConsts<double>& c, hipStream_t s) {
  const bool ph = L.wtab != nullptr;
  if (ph) {
    return L.strain ? launch_t<T, TO, TW, true, true>(L, c, s)
                    : launch_t<T, TO, TW, true, false>(L, c, s);
  }
  return L.strain ? launch_t<T, TO, TW, false, true>(L, c, s)
                  : launch_t<T, TO, TW, false, false>(L, c, s);
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
    return launch_ph<double, double, double>(L, c, s);
  }
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
