// Two steps of the Chebyshev recurrence of the filter (paper Sec. II.B) in one
// pass over the grid (temporal blocking):
//
//     Y1 = alpha1 (H - shift1) Y0 + beta1 Y_old
//     Y2 = alpha2 (H - shift2) Y1 + beta2 Y0
//
// with H the finite-difference hole Hamiltonian of Eq. HNI, complex FP32.  One
// step reads two blocks and writes one; this pass reads two (Y0, Y_old) and
// writes two (Y1, Y2), so the filter moves 2 blocks per step instead of 3.
//
// Kernel design (gfx950).  A workgroup owns a TX x TY tile of (x, y) columns of
// one vector and marches along z.  Every plane of Y0 is staged in LDS with a
// two-point halo ring, (TX + 4) x (TY + 4) per component, by global -> LDS
// copies (16 bytes per lane, no registers) issued one plane ahead.  Step one
// runs on the tile plus a one-point ring, (TX + 2) x (TY + 2) columns, with the
// arithmetic of the one-step kernel (contributions of each input plane pushed
// into register accumulators of the output planes below, at and above it);
// every finished plane of Y1 goes to an LDS plane (zero outside the grid: hard
// wall) and, on the tile's own columns, to HBM.  Step two reads that LDS plane
// with the same push arithmetic on the tile's columns and writes Y2.  The ring
// costs (TX + 2)(TY + 2) / (TX TY) of step one's arithmetic (1.31 for 16 x 12)
// and saves a third of the filter's HBM traffic.  Threads map 2D patches (one
// spin per wave), so TX is not tied to the 64-lane wave and the tile can match
// the grid; x needs nx % TX == 0 (whole 16-byte pairs of points in the rows).
//
// Y1 and Y2 must not overwrite Y0 or Y_old: workgroups read both on their halo
// rings, which neighbouring workgroups own.  Used for B = 0 and for fields with
// Bz = 0 (link phases uniform over each z-plane).
#include "hkp_internal.h"
#include "stencil_ops.h"

namespace hkp {

namespace {

using namespace sten;

struct K2Args {
  const float* in;     // Y0
  const float* old;    // Y_old
  float* out1;         // Y1
  float* out2;         // Y2
  long long bstride;   // complex elements between members (all four blocks)
  const float* D;
  long long D_bstride;
  const float* zero;   // 16 bytes of zeros in device memory (the wall's values)
  const float* wtab;   // [nz] x-link phases (complex)
  const float* vtab;   // [nz][nx] y-link phases (complex; uniform over x here)
  const double* coef1;   // per member [alpha, shift, beta] of the first step, or null:
  const double* coef2;   // the host values below; and of the second
  int coef_stride;
  double h1[3], h2[3];   // host alpha, shift, beta of the two steps
  const int* active;
  const int* lock;
  const int* work;
  int batch;
  int nx, ny, nz, nvec;
  int tiles_x, tiles_y;
  int vgroup;
  StencilConsts<float> k;
};

constexpr int round64(int n) { return (n + 63) / 64 * 64; }

template <int PH, bool STR, int TX, int TY>
__global__ void __launch_bounds__(2 * round64((TX + 2) * (TY + 2)))
stencil2_kernel(K2Args a) {
  static_assert(PH == 0 || PH == 1, "link phases uniform over each z-plane only");
  static_assert(TX % 2 == 0, "rows are copied in 16-byte pairs of points");
  using T = float;
  constexpr int EW = TX + 2, EH = TY + 2;   // step one: tile + one-point ring
  constexpr int E = EW * EH;
  constexpr int EP = round64(E);            // threads per spin
  constexpr int NT = 2 * EP;
  constexpr int O = TX * TY;                // step two: the tile
  static_assert(O <= EP, "step two maps into the threads of step one");
  constexpr int IW = TX + 4, IH = TY + 4;   // Y0 plane: tile + two-point ring
  constexpr int IPL = IW * IH;
  constexpr int EPL = E;
  constexpr int CPR = IW / 2;               // 16-byte chunks per row
  constexpr int NCH = 6 * IH * CPR;         // chunks per plane
  constexpr int NR = (NCH + NT - 1) / NT;   // copy rounds per plane
  // Y0 planes, padded to the copy rounds' chunks (lanes past the plane copy zeros
  // into the padding)
  __shared__ cx<T> y0a[2 * NR * NT];
  __shared__ cx<T> y0b[2 * NR * NT];
  __shared__ cx<T> y1a[6 * EPL];
  __shared__ cx<T> y1b[6 * EPL];
  auto bufp = [&](auto BUF) -> cx<T>* {
    if constexpr (decltype(BUF)::value == 0) return y0a; else return y0b;
  };
  auto buf1 = [&](auto BUF) -> cx<T>* {
    if constexpr (decltype(BUF)::value == 0) return y1a; else return y1b;
  };

  // ---- workgroup -> (member, vector, tile); the order of the one-step kernel
  const int ntiles = a.tiles_x * a.tiles_y;
  int b, vec, tile;
  if (a.work) {
    const int nv = a.work[a.batch];
    const int nlive = nv * ntiles;
    if ((int)blockIdx.x >= nlive) return;
    const int logical = xcd_remap(blockIdx.x, nlive);
    const int g = logical / (a.vgroup * ntiles);
    const int within = logical - g * a.vgroup * ntiles;
    const int gsize = min(a.vgroup, nv - g * a.vgroup);
    tile = within / gsize;
    const int u = g * a.vgroup + (within - tile * gsize);
    b = 0;
    while (a.work[b + 1] <= u) ++b;
    vec = (a.lock ? a.lock[b] : 0) + (u - a.work[b]);
  } else {
    const int nlive = (int)gridDim.x;
    const int logical = xcd_remap(blockIdx.x, nlive);
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
  const int x0 = (tile % a.tiles_x) * TX;
  const int y0 = (tile / a.tiles_x) * TY;

  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const unsigned nxy = (unsigned)nx * (unsigned)ny;
  const unsigned N = nxy * (unsigned)nz;   // 6 N < 2^31 (checked on the host)
  const int t = threadIdx.x;
  const int sp = __builtin_amdgcn_readfirstlane(t / EP);   // spin: uniform per wave
  const int e = t - sp * EP;
  const int X = 3 * sp, F = 3 - X;

  // step-one column (tile + ring) and step-two column (tile) of this thread
  const bool v1 = e < E;
  const int ey = v1 ? e / EW : 0, ex = v1 ? e - (e / EW) * EW : 0;
  const int gx1 = x0 - 1 + ex, gy1 = y0 - 1 + ey;
  const bool in1 = v1 && gx1 >= 0 && gx1 < nx && gy1 >= 0 && gy1 < ny;
  const bool own1 = in1 && ex >= 1 && ex <= TX && ey >= 1 && ey <= TY;
  const unsigned col1 = in1 ? (unsigned)(gy1 * nx + gx1) : 0u;
  const int lb1 = (ey + 1) * IW + (ex + 1);   // centre in a Y0 plane
  const int ly1 = ey * EW + ex;               // slot in the Y1 plane
  const bool v2 = e < O;
  const int oy = v2 ? e / TX : 0, ox = v2 ? e - (e / TX) * TX : 0;
  const int gx2 = x0 + ox, gy2 = y0 + oy;
  const bool in2 = v2 && gx2 < nx && gy2 < ny;
  const unsigned col2 = in2 ? (unsigned)(gy2 * nx + gx2) : 0u;
  const int lb2 = (oy + 1) * EW + (ox + 1);   // centre in the Y1 plane
  const int lk2 = (oy + 2) * IW + (ox + 2);   // same column in a Y0 plane

  T alpha1 = (T)a.h1[0], shift1 = (T)a.h1[1], beta1 = (T)a.h1[2];
  T alpha2 = (T)a.h2[0], shift2 = (T)a.h2[1], beta2 = (T)a.h2[2];
  if (a.coef1) {
    const double* c1 = a.coef1 + (long long)b * a.coef_stride;
    const double* c2 = a.coef2 + (long long)b * a.coef_stride;
    alpha1 = (T)c1[0];
    shift1 = (T)c1[1];
    beta1 = (T)c1[2];
    alpha2 = (T)c2[0];
    shift2 = (T)c2[1];
    beta2 = (T)c2[2];
  }
  const bool has_old = beta1 != (T)0;

  const long long vb = (long long)b * a.bstride + (long long)vec * 6 * N;   // complex elements
  const T* __restrict__ in = a.in + 2 * vb;
  const T* __restrict__ oldp = a.old + 2 * (vb + (long long)X * N);
  T* __restrict__ o1 = a.out1 + 2 * (vb + (long long)X * N);
  T* __restrict__ o2 = a.out2 + 2 * (vb + (long long)X * N);
  const T* __restrict__ D = a.D + (long long)b * a.D_bstride;
  const StencilConsts<T> k = a.k;
  const T dgs = sp == 0 ? k.dgU : k.dgD;
  const T ax = sp == 0 ? k.aUx : k.aDx, ay = sp == 0 ? k.aUy : k.aDy,
          az = sp == 0 ? k.aUz : k.aDz;
  const T sd3 = sp == 0 ? -k.d3 : k.d3;
  const T sby = sp == 0 ? -k.by : k.by;

  // ---- Y0 plane copies: chunk q of a plane is 16 bytes (two points) of row
  // (component, iy) at column pair ic, and lands at byte 16 q of the LDS plane.
  // Chunks outside the grid (and lanes past the plane) copy 16 zero bytes from
  // a.zero: every lane of every wave issues the same copies, with no branch,
  // so that waits for the loads issued before them never wait for the copies.
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  unsigned coff[NR];
  bool cval[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int q = t + NT * r;
    const int c = q / (IH * CPR), rem = q - c * (IH * CPR);
    const int iy = rem / CPR, ic = rem - iy * CPR;
    const int gy = y0 - 2 + iy, gx = x0 - 2 + 2 * ic;
    cval[r] = q < NCH && gy >= 0 && gy < ny && gx >= 0 && gx + 1 < nx;
    coff[r] = cval[r] ? (unsigned)c * N + (unsigned)(gy * nx + gx) : 0u;
  }
  auto copy_plane = [&](int z, auto BUF) {
    cx<T>* dst = bufp(BUF);
    const unsigned zo = (unsigned)z * nxy;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const T* src = cval[r] ? in + 2 * (size_t)(coff[r] + zo) : a.zero;
      dma16(src, dst + 2 * (NT * r + 64 * wave));
    }
  };

  // ---- phases (uniform over a plane) and on-site fields, one plane ahead
  constexpr int ND = STR ? 6 : 1;
  auto load_d = [&](int z, unsigned col, T (&d)[ND]) {
    const unsigned pz = (unsigned)z * nxy + col;
#pragma unroll
    for (int i = 0; i < ND; ++i) d[i] = D[(unsigned)i * N + pz];
  };
  auto wph = [&](int z) { return ld(a.wtab + 2 * (z < 0 ? 0 : (z >= nz ? nz - 1 : z))); };
  auto vph = [&](int z) {
    return ld(a.vtab + 2 * (size_t)((z < 0 ? 0 : (z >= nz ? nz - 1 : z)) * nx));
  };
  // step one pushes Y0 plane z, step two Y1 plane z - 2: windows of planes
  // (z-1, z, z+1) and (z-3, z-2, z-1) at iteration z
  cx<T> pw1[3], pv1[3], pw2[3], pv2[3];
  const cx<T> zero = mk<T>(0, 0);
#pragma unroll
  for (int i = 0; i < 3; ++i) pw1[i] = pv1[i] = pw2[i] = pv2[i] = zero;
  if constexpr (PH != 0) {
    pw1[0] = wph(-1); pw1[1] = wph(0); pw1[2] = wph(1);
    pv1[0] = vph(-1); pv1[1] = vph(0); pv1[2] = vph(1);
    pw2[0] = wph(-3); pw2[1] = wph(-2); pw2[2] = wph(-1);
    pv2[0] = vph(-3); pv2[1] = vph(-2); pv2[2] = vph(-1);
  }

  // accumulators of Y1 planes z-1, z, z+1 (acc) and of Y2 planes z-3, z-2,
  // z-1 (bcc); this column's Y0 of planes z-3, z-2, z-1 for the beta term of Y2
  cx<T> acc0[3], acc1[3], acc2[3], bcc0[3], bcc1[3], bcc2[3], oldv[3];
  cx<T> ka[3], kb[3], kc[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    acc0[i] = acc1[i] = acc2[i] = bcc0[i] = bcc1[i] = bcc2[i] = oldv[i] = zero;
    ka[i] = kb[i] = kc[i] = zero;
  }
  T d1[ND], d2[ND];
  load_d(0, col1, d1);
#pragma unroll
  for (int i = 0; i < ND; ++i) d2[i] = (T)0;

  copy_plane(0, IC<0>{});
  __syncthreads();

  // iteration z: step one on Y0 plane z (buffer z & 1) completes Y1 plane z - 1
  // (to Y1 buffer (z - 1) & 1); step two on Y1 plane z - 2 (buffer z & 1, written
  // in the previous iteration) completes Y2 plane z - 3.  One barrier per plane.
  auto iteration = [&](int z, auto BUF) {
    constexpr int cur = decltype(BUF)::value;
    // loads in the order they are needed (the memory counter retires them in
    // order, so a wait for an early load does not wait for the copy of the next
    // plane): fields and phases for the next iteration, the old block for
    // Y1(z-1) (column 0 for threads off the grid: no branch), then the next
    // Y0 plane's rows into the other buffer
    T n1[ND], n2[ND];
    load_d(z + 1 < nz ? z + 1 : nz - 1, col1, n1);
    load_d(z - 1 < 0 ? 0 : (z - 1 < nz ? z - 1 : nz - 1), col2, n2);
    cx<T> nw1 = zero, nv1 = zero, nw2 = zero, nv2 = zero;
    if constexpr (PH != 0) {
      nw1 = wph(z + 2);
      nv1 = vph(z + 2);
      nw2 = wph(z);
      nv2 = vph(z);
    }
    {   // read even when beta1 == 0 (a valid block; the value is then unused)
      const int zo = z - 1 < 0 ? 0 : (z - 1 < nz ? z - 1 : nz - 1);
      const unsigned o = (unsigned)zo * nxy + col1;
#pragma unroll
      for (int i = 0; i < 3; ++i) oldv[i] = ld_stream(oldp + 2 * (size_t)((unsigned)i * N + o));
    }
    // past the last plane the copy repeats it into the buffer no longer read
    copy_plane(z + 1 < nz ? z + 1 : nz - 1, IC<1 - cur>{});

    // ---- step one: push Y0 plane z (tile + ring)
    if (z < nz) {
      const cx<T>* L = bufp(IC<cur>{}) + lb1;
      const T d00 = d1[0], d11 = d1[STR ? 1 : 0], d22 = d1[STR ? 2 : 0];
      const T d12 = STR ? d1[STR ? 3 : 0] : (T)0;
      const T d02 = STR ? d1[STR ? 4 : 0] : (T)0;
      const T d01 = STR ? d1[STR ? 5 : 0] : (T)0;
      push_plane<T, PH, STR, 6, IPL, IW>(L, X, F, k, dgs, ax, ay, az, sd3, sby, shift1, pw1,
                                         pv1, zero, zero, d00, d11, d22, d12, d02, d01, acc0,
                                         acc1, acc2);
    }
    // this thread's tile column of Y0 plane z (own spin), for Y2's beta term
    cx<T> kd[3];
    {
      const cx<T>* K = bufp(IC<cur>{}) + lk2;
#pragma unroll
      for (int i = 0; i < 3; ++i) kd[i] = K[(X + i) * IPL];
    }
    // ---- step two: push Y1 plane z - 2 (tile)
    const bool s2 = z >= 2 && z - 2 < nz;
    if (s2) {
      const cx<T>* L = buf1(IC<cur>{}) + lb2;
      const T d00 = d2[0], d11 = d2[STR ? 1 : 0], d22 = d2[STR ? 2 : 0];
      const T d12 = STR ? d2[STR ? 3 : 0] : (T)0;
      const T d02 = STR ? d2[STR ? 4 : 0] : (T)0;
      const T d01 = STR ? d2[STR ? 5 : 0] : (T)0;
      push_plane<T, PH, STR, 6, EPL, EW>(L, X, F, k, dgs, ax, ay, az, sd3, sby, shift2, pw2,
                                         pv2, zero, zero, d00, d11, d22, d12, d02, d01, bcc0,
                                         bcc1, bcc2);
    }
    // both steps' arithmetic is done before the stores below: their wait for the
    // old block also waits for the next plane's copy, which is then in flight
    // during all of it (the Y1 plane goes to the buffer step two does not read)
    settle(acc1);
    settle(acc2);
    settle(bcc1);
    settle(bcc2);
    // ---- Y1 plane z - 1 is complete: to LDS (zero off the grid) and HBM
    if (z >= 1 && z - 1 < nz && v1) {
      cx<T>* Y1 = buf1(IC<1 - cur>{});
      const unsigned o = (unsigned)(z - 1) * nxy + col1;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        cx<T> r = scl(alpha1, acc0[i]);
        if (has_old) r = fma_s(r, beta1, oldv[i]);
        if (!in1) r = zero;
        Y1[(X + i) * EPL + ly1] = r;
        if (own1) stg_stream<T>(o1, (long long)((unsigned)i * N + o), r);
      }
    }
    if (z < nz) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        acc0[i] = acc1[i];
        acc1[i] = acc2[i];
      }
    }

    // ---- Y2 plane z - 3 is complete
    if (z >= 3 && in2) {
      const unsigned o = (unsigned)(z - 3) * nxy + col2;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        cx<T> r = scl(alpha2, bcc0[i]);
        r = fma_s(r, beta2, ka[i]);
        stg_stream<T>(o2, (long long)((unsigned)i * N + o), r);
      }
    }
    if (s2) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        bcc0[i] = bcc1[i];
        bcc1[i] = bcc2[i];
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      ka[i] = kb[i];
      kb[i] = kc[i];
      kc[i] = kd[i];
    }
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      d1[i] = n1[i];
      d2[i] = n2[i];
    }
    if constexpr (PH != 0) {
      pw1[0] = pw1[1]; pw1[1] = pw1[2]; pw1[2] = nw1;
      pv1[0] = pv1[1]; pv1[1] = pv1[2]; pv1[2] = nv1;
      pw2[0] = pw2[1]; pw2[1] = pw2[2]; pw2[2] = nw2;
      pv2[0] = pv2[1]; pv2[1] = pv2[2]; pv2[2] = nv2;
    }
    __syncthreads();   // next Y0 plane copied; Y1 plane z - 1 published; buffers retired
  };

  for (int z = 0; z <= nz + 2; z += 2) {
    iteration(z, IC<0>{});
    if (z + 1 <= nz + 2) iteration(z + 1, IC<1>{});
  }
}

template <int PH, bool STR>
hipError_t launch_ts(const K2Args& a, int tx, int ty, hipStream_t s) {
  const long long nwg = (long long)a.tiles_x * a.tiles_y * a.nvec * a.batch;
  if (nwg <= 0) return hipSuccess;
  if (nwg > 0x7fffffffLL) return hipErrorInvalidValue;
  auto go = [&](auto kernel, int threads) {
    kernel<<<dim3((unsigned)nwg), dim3(threads), 0, s>>>(a);
  };
  if (tx == 16 && ty == 12) go(stencil2_kernel<PH, STR, 16, 12>, 2 * round64(18 * 14));
  else if (tx == 16 && ty == 8) go(stencil2_kernel<PH, STR, 16, 8>, 2 * round64(18 * 10));
  else if (tx == 32 && ty == 8) go(stencil2_kernel<PH, STR, 32, 8>, 2 * round64(34 * 10));
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

bool stencil2_supported(const Stencil2Launch& L) {
  const bool shape = (L.tile_x == 16 && (L.tile_y == 12 || L.tile_y == 8)) ||
                     (L.tile_x == 32 && L.tile_y == 8);
  return shape && L.nx % L.tile_x == 0 && !L.phase_general;
}

hipError_t launch_stencil2(const Stencil2Launch& L, const StencilConsts<double>& c,
                           hipStream_t s) {
  if (!stencil2_supported(L) || (!L.coef1) != (!L.coef2) || !L.zero) return hipErrorInvalidValue;
  K2Args a;
  for (int i = 0; i < 3; ++i) {
    a.h1[i] = L.host1[i];
    a.h2[i] = L.host2[i];
  }
  a.in = static_cast<const float*>(L.in);
  a.old = static_cast<const float*>(L.old);
  a.out1 = static_cast<float*>(L.out1);
  a.out2 = static_cast<float*>(L.out2);
  a.bstride = L.bstride;
  a.D = static_cast<const float*>(L.D);
  a.D_bstride = L.D_bstride;
  a.zero = static_cast<const float*>(L.zero);
  a.wtab = static_cast<const float*>(L.wtab);
  a.vtab = static_cast<const float*>(L.vtab);
  a.coef1 = L.coef1;
  a.coef2 = L.coef2;
  a.coef_stride = L.coef_stride;
  a.active = L.active;
  a.lock = L.lock;
  a.work = L.work;
  a.batch = L.batch;
  a.nx = L.nx;
  a.ny = L.ny;
  a.nz = L.nz;
  a.nvec = L.nvec;
  a.tiles_x = L.nx / L.tile_x;
  a.tiles_y = (L.ny + L.tile_y - 1) / L.tile_y;
  a.vgroup = L.vgroup < 1 ? 1 : (L.vgroup > L.nvec ? L.nvec : L.vgroup);
  a.k = cast_consts<float>(c);
  const bool field = L.wtab != nullptr;
  if (field) return L.strain ? launch_ts<1, true>(a, L.tile_x, L.tile_y, s)
                             : launch_ts<1, false>(a, L.tile_x, L.tile_y, s);
  return L.strain ? launch_ts<0, true>(a, L.tile_x, L.tile_y, s)
                  : launch_ts<0, false>(a, L.tile_x, L.tile_y, s);
}

}  // namespace hkp
