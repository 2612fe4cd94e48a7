// Complex helpers and the per-plane arithmetic of the finite-difference hole
// Hamiltonian in the |L S> basis (paper Eq. LK, with the Bir-Pikus, Zeeman and
// Peierls terms of Eq. HNI), shared by the one-step and the two-step stencil
// kernels.  Device code only; included by the stencil sources.
#pragma once

#include "hkp_internal.h"

namespace hkp {
namespace sten {

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
// acc + c a + conj(c) b  (c carries a real stencil coefficient times a link phase)
template <typename T>
__device__ __forceinline__ cx<T> wsum_acc(cx<T> acc, cx<T> c, cx<T> a, cx<T> b) {
  cx<T> d = sub(a, b), s = add(a, b);
  return {fma(-c.i, d.i, fma(c.r, s.r, acc.r)), fma(c.i, d.r, fma(c.r, s.i, acc.i))};
}
// acc + c a - conj(c) b
template <typename T>
__device__ __forceinline__ cx<T> wdiff_acc(cx<T> acc, cx<T> c, cx<T> a, cx<T> b) {
  cx<T> d = sub(a, b), s = add(a, b);
  return {fma(-c.i, s.i, fma(c.r, d.r, acc.r)), fma(c.i, s.r, fma(c.r, d.i, acc.i))};
}

template <typename T>
__device__ __forceinline__ cx<T> ld(const T* p) {
  typename V2<T>::type v = *reinterpret_cast<const typename V2<T>::type*>(p);
  return {v.x, v.y};
}
template <typename TW, typename T>
__device__ __forceinline__ void stg(void* base, long long idx, cx<T> v) {
  typename V2<TW>::type o;
  o.x = static_cast<TW>(v.r);
  o.y = static_cast<TW>(v.i);
  reinterpret_cast<typename V2<TW>::type*>(base)[idx] = o;
}

// Streams touched once per launch (the previous iterate, the output) go through
// the cache with the non-temporal policy, so that they do not push the on-site
// fields and the input rows, which later workgroups of the same XCD reuse, out
// of the L2.
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
template <typename T> struct NT2;
template <> struct NT2<float> { using type = nt_f2; };
template <> struct NT2<double> { using type = nt_d2; };
template <typename T>
__device__ __forceinline__ cx<T> ld_stream(const T* p) {
  const typename NT2<T>::type v =
      __builtin_nontemporal_load(reinterpret_cast<const typename NT2<T>::type*>(p));
  return {v.x, v.y};
}
template <typename TW, typename T>
__device__ __forceinline__ void stg_stream(void* base, long long idx, cx<T> v) {
  typename NT2<TW>::type o;
  o.x = static_cast<TW>(v.r);
  o.y = static_cast<TW>(v.i);
  __builtin_nontemporal_store(o, reinterpret_cast<typename NT2<TW>::type*>(base) + idx);
}



// 16 bytes per lane, global -> LDS without registers: lane t's bytes land at
// lds + 16 t (lds is wave-uniform).  The builtin exists only for the device
// pass; the host pass sees an empty body so the kernel's host stub is emitted.
__device__ __forceinline__ void dma16(const void* g, void* lds) {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
#endif
}

// Ends the computation of these accumulators here: an empty asm statement that
// takes them as register inputs (it emits nothing), placed before a plane's
// output stores, stops the compiler from sinking this plane's arithmetic past
// the stores.  The stores need the old block, and the wait for it also waits for
// the next plane's copy issued after it; with the arithmetic done first, that
// copy is in flight during all of it.
template <typename T>
__device__ __forceinline__ void settle(const cx<T> (&a)[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) asm volatile("" ::"v"(a[i].r), "v"(a[i].i));
}

template <int V>
struct IC {
  static constexpr int value = V;
};

// Contributions of one input plane z of one spin's three orbital components
// (this thread's column; the plane sits in LDS as [component][row][column] with
// plane stride PLANE and row width W, L pointing at this column's centre) to
// the output planes z-1 (added to acc0), z (added to acc1) and z+1 (written to
// acc2).  X / F: component offsets of this thread's spin and of the other one.
// pw, pv: x- and y-link phases of planes z-1, z, z+1; pvxp, pvxm: the y-links of
// the neighbouring columns in plane z (PH == 2).  d..: the on-site orbital block
// of this column at plane z.  In-plane terms (faces, x-y edges, on-site,
// spin-orbit and Zeeman) go to plane z; the z faces and the x-z / y-z edges of
// the plane are pushed to z-1 and z+1.
template <typename T, int PH, bool STR, int NC, int PLANE, int W>
__device__ __forceinline__ void push_plane(
    const cx<T>* L, int X, int F, const StencilConsts<T>& k, T dgs, T ax, T ay, T az, T sd3,
    T sby, T shift, const cx<T> (&pw)[3], const cx<T> (&pv)[3], cx<T> pvxp, cx<T> pvxm,
    T d00, T d11, T d22, T d12, T d02, T d01, cx<T> (&acc0)[3], cx<T> (&acc1)[3],
    cx<T> (&acc2)[3]) {
  auto at = [&](int c, int dy, int dx) { return L[c * PLANE + dy * W + dx]; };

  // ---- phases (GPU gauge): x-links per plane, y-links per (plane, column);
  // with Bz = 0 (PH == 1) every phase is uniform over the plane
  const cx<T> wm = pw[0], w0 = pw[1], wp = pw[2], vm = pv[0], v0 = pv[1], vp = pv[2];
  const cx<T> vxp = pvxp, vxm = pvxm;

  {
    // faces in the plane (this spin's three orbitals); the coefficient of the
    // x faces is (L-M) + M on |X> and M on |Y>, |Z> (y faces: on |Y> and the
    // others), folded with the link phase into one complex constant per plane
    const T cLMM = k.cLM + k.cM;
    if constexpr (PH != 0) {
      const cx<T> cx_o = scl(k.cM, w0), cx_a = scl(cLMM, w0);
      const cx<T> cy_o = scl(k.cM, v0), cy_a = scl(cLMM, v0);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        acc1[i] = wsum_acc(acc1[i], i == 0 ? cx_a : cx_o, at(X + i, 0, 1), at(X + i, 0, -1));
        acc1[i] = wsum_acc(acc1[i], i == 1 ? cy_a : cy_o, at(X + i, 1, 0), at(X + i, -1, 0));
      }
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const cx<T> sx = add(at(X + i, 0, 1), at(X + i, 0, -1));
        const cx<T> sy = add(at(X + i, 1, 0), at(X + i, -1, 0));
        acc1[i] = fma_s(acc1[i], i == 0 ? cLMM : k.cM, sx);
        acc1[i] = fma_s(acc1[i], i == 1 ? cLMM : k.cM, sy);
      }
    }
  }
  {
    // x-y edges (in plane): couple X <-> Y
    const cx<T> fY_pp = at(X + 1, 1, 1), fY_pm = at(X + 1, -1, 1);
    const cx<T> fY_mp = at(X + 1, 1, -1), fY_mm = at(X + 1, -1, -1);
    const cx<T> fX_pp = at(X, 1, 1), fX_pm = at(X, -1, 1);
    const cx<T> fX_mp = at(X, 1, -1), fX_mm = at(X, -1, -1);
    if constexpr (PH == 2) {
      // P(sx, sy) = w^sx [ v(x+sx)^sy + v(x)^sy ]
      const cx<T> ppp = mul(w0, add(vxp, v0));
      const cx<T> ppm = mul(w0, conj(add(vxp, v0)));
      const cx<T> pmp = mul(conj(w0), add(vxm, v0));
      const cx<T> pmm = mul(conj(w0), conj(add(vxm, v0)));
      cx<T> eY = sub(add(mul(ppp, fY_pp), mul(pmm, fY_mm)), add(mul(ppm, fY_pm), mul(pmp, fY_mp)));
      cx<T> eX = sub(add(mul(ppp, fX_pp), mul(pmm, fX_mm)), add(mul(ppm, fX_pm), mul(pmp, fX_mp)));
      acc1[0] = fma_s(acc1[0], k.cN8, eY);
      acc1[1] = fma_s(acc1[1], k.cN8, eX);
    } else if constexpr (PH == 1) {
      // uniform phases: P(sx, sy) = 2 w^sx v^sy, so the corner sum is
      // q f++ + conj(q) f-- - (p f+- + conj(p) f-+) with q = 2 cN8 w v and
      // p = 2 cN8 w conj(v) (f indexed by the signs of dx, dy)
      const T c2 = k.cN8 + k.cN8;
      const cx<T> q = scl(c2, mul(w0, v0)), mp = scl(-c2, mul(w0, conj(v0)));
      acc1[0] = wsum_acc(wsum_acc(acc1[0], q, fY_pp, fY_mm), mp, fY_pm, fY_mp);
      acc1[1] = wsum_acc(wsum_acc(acc1[1], q, fX_pp, fX_mm), mp, fX_pm, fX_mp);
    } else {
      cx<T> eY = sub(add(fY_pp, fY_mm), add(fY_pm, fY_mp));
      cx<T> eX = sub(add(fX_pp, fX_mm), add(fX_pm, fX_mp));
      const T c2 = k.cN8 + k.cN8;
      acc1[0] = fma_s(acc1[0], c2, eY);
      acc1[1] = fma_s(acc1[1], c2, eX);
    }
  }
  {
    const cx<T> oX = at(X, 0, 0), oY = at(X + 1, 0, 0), oZ = at(X + 2, 0, 0);
    // z faces: pushed to z-1 and z+1
    acc0[0] = fma_s(acc0[0], k.cM, oX);
    acc0[1] = fma_s(acc0[1], k.cM, oY);
    acc0[2] = fma_s(acc0[2], k.czZ, oZ);
    acc2[0] = scl(k.cM, oX);
    acc2[1] = scl(k.cM, oY);
    acc2[2] = scl(k.czZ, oZ);
    // x-z and y-z edges of this plane, pushed to z-1 (sz = +1) and z+1 (sz = -1)
    const cx<T> xpZ = at(X + 2, 0, 1), xmZ = at(X + 2, 0, -1);
    const cx<T> xpX = at(X, 0, 1), xmX = at(X, 0, -1);
    const cx<T> ypZ = at(X + 2, 1, 0), ymZ = at(X + 2, -1, 0);
    const cx<T> ypY = at(X + 1, 1, 0), ymY = at(X + 1, -1, 0);
    if constexpr (PH != 0) {
      // path-averaged phases (x2) times +-cN8, one complex constant each
      const cx<T> cu = scl(k.cN8, add(wm, w0)), cd = scl(-k.cN8, add(wp, w0));
      const cx<T> du = scl(k.cN8, add(vm, v0)), dd = scl(-k.cN8, add(vp, v0));
      acc0[0] = wdiff_acc(acc0[0], cu, xpZ, xmZ);
      acc0[2] = wdiff_acc(wdiff_acc(acc0[2], cu, xpX, xmX), du, ypY, ymY);
      acc0[1] = wdiff_acc(acc0[1], du, ypZ, ymZ);
      acc2[0] = wdiff_acc(acc2[0], cd, xpZ, xmZ);
      acc2[2] = wdiff_acc(wdiff_acc(acc2[2], cd, xpX, xmX), dd, ypY, ymY);
      acc2[1] = wdiff_acc(acc2[1], dd, ypZ, ymZ);
    } else {
      const T c2 = k.cN8 + k.cN8;
      const cx<T> dxZ = sub(xpZ, xmZ), dxX = sub(xpX, xmX);
      const cx<T> dyZ = sub(ypZ, ymZ), dyY = sub(ypY, ymY);
      acc0[0] = fma_s(acc0[0], c2, dxZ);
      acc0[2] = fma_s(acc0[2], c2, add(dxX, dyY));
      acc0[1] = fma_s(acc0[1], c2, dyZ);
      acc2[0] = fma_s(acc2[0], -c2, dxZ);
      acc2[2] = fma_s(acc2[2], -c2, add(dxX, dyY));
      acc2[1] = fma_s(acc2[1], -c2, dyZ);
    }

    // ---- on-site: orbital block (V + strain), constants, SO/Zeeman
    const T dg = dgs - shift;
    cx<T> r0v = scl(d00 + dg, oX), r1v = scl(d11 + dg, oY), r2v = scl(d22 + dg, oZ);
    if constexpr (STR) {
      r0v = fma_s(fma_s(r0v, d01, oY), d02, oZ);
      r1v = fma_s(fma_s(r1v, d01, oX), d12, oZ);
      r2v = fma_s(fma_s(r2v, d02, oX), d12, oY);
    }
    // i (a x u)
    if constexpr (PH != 0) {
      r0v = add(r0v, mul_i(sub(scl(ay, oZ), scl(az, oY))));
      r1v = add(r1v, mul_i(sub(scl(az, oX), scl(ax, oZ))));
      r2v = add(r2v, mul_i(sub(scl(ax, oY), scl(ay, oX))));
    } else {
      r0v = fma_s(r0v, -az, mul_i(oY));
      r1v = fma_s(r1v, az, mul_i(oX));
    }
    // spin flip: up <- -d3 (v_Z, -i v_Z, -v_X + i v_Y) + (bx - i by) v   (v = down)
    //            dn <- -d3 (-v_Z, -i v_Z, v_X + i v_Y) + (bx + i by) v   (v = up)
    // i.e. r_X += s d3 v_Z, r_Y += d3 i v_Z, r_Z += -d3 i v_Y - s d3 v_X with
    // s = -1 (up), +1 (down)
    if constexpr (NC == 6) {   // spin-free vectors have no other spin to couple to
      const cx<T> f0 = at(F, 0, 0), f1 = at(F + 1, 0, 0), f2 = at(F + 2, 0, 0);
      r0v = fma_s(r0v, sd3, f2);
      r1v = fma_s(r1v, k.d3, mul_i(f2));
      r2v = fma_s(fma_s(r2v, -k.d3, mul_i(f1)), -sd3, f0);
      if constexpr (PH != 0) {
        const cx<T> bz = mk<T>(k.bx, sby);
        r0v = add(r0v, mul(bz, f0));
        r1v = add(r1v, mul(bz, f1));
        r2v = add(r2v, mul(bz, f2));
      }
    }
    acc1[0] = add(acc1[0], r0v);
    acc1[1] = add(acc1[1], r1v);
    acc1[2] = add(acc1[2], r2v);
  }
}

}  // namespace sten
}  // namespace hkp
