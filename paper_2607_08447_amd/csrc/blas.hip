// Block operations of the subspace iteration on tall-skinny complex blocks
// X (n x nb, vector-major: each vector contiguous, complex interleaved):
//
//   Gram     C = A^H B (nb x nb)          FP64 MFMA (v_mfma_f64_16x16x4f64),
//                                         split over K, fixed-order reduction
//   rotate   X <- X Q                     FP64 MFMA, in place
//   Ritz     W Q, not stored: r_j^2 = || (W Q)_j - theta_j (X Q)_j ||^2 and the
//            first filter step Y1 = alpha (W Q - shift X Q)
//   Lanczos  dots, three-term update, normalisation (spectral bound)
//
// The complex products are evaluated as real products of the (re, im)
// columns: Re(A^H B) = Ar'Br + Ai'Bi, Im(A^H B) = Ar'Bi - Ai'Br, so the
// MFMA work equals the complex flop count (8 n nb^2 real flops per product).
#include "hkp_internal.h"

namespace hkp {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kGramChunkMin = 1024;   // complex elements per split-K chunk, minimum

// ---------------------------------------------------------------------------
// Gram: one wave per 16-vector row tile of A; it walks every 16-vector column
// tile of B (only j >= i for a Hermitian product).  MFMA operand layout for
// 16x16x4 f64: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; the
// result D[i][j] sits in lane j + 16 (i % 4), register i / 4 (checked on gfx950).
// ---------------------------------------------------------------------------
template <int NT>
__global__ void __launch_bounds__(64 * 4)
gram_partial_kernel(const double* A, long long a_bstride, int nba, const double* B,
                    long long b_bstride, int nbb, long long n, long long chunk, int hermitian,
                    const int* active, double* partial) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ti = blockIdx.y * 4 + wv;   // row tile handled by this wave
  const int b = blockIdx.z;
  const int nchunks = gridDim.x;
  if (active && !active[b]) return;
  const int ntb = (nbb + 15) / 16;
  if (ti * 16 >= nba) return;
  const long long e0 = (long long)blockIdx.x * chunk;
  long long e1 = e0 + chunk;
  if (e1 > n) e1 = n;
  const int r = lane & 15, q = lane >> 4;
  const int va = ti * 16 + r;
  const bool vaok = va < nba;
  const double* pa = A + 2 * ((long long)b * a_bstride + (long long)(vaok ? va : 0) * n);
  const double* pb[NT];
  bool vbok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int vb = t * 16 + r;
    vbok[t] = t < ntb && vb < nbb;
    pb[t] = B + 2 * ((long long)b * b_bstride + (long long)(vbok[t] ? vb : 0) * n);
  }
  d4 rr[NT], ii[NT], ri[NT], ir[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    rr[t] = d4{0, 0, 0, 0};
    ii[t] = rr[t];
    ri[t] = rr[t];
    ir[t] = rr[t];
  }
  const int t0 = hermitian ? ti : 0;
  const long long nks = (e1 - e0 + 3) / 4;   // k-steps (uniform across the wave)
  for (long long st = 0; st < nks; ++st) {
    const long long e = e0 + 4 * st + q;
    const bool eok = e < e1;
    double2 av = (vaok && eok) ? *reinterpret_cast<const double2*>(pa + 2 * e) : make_double2(0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (t < t0 || t >= ntb) continue;
      double2 bv = (vbok[t] && eok) ? *reinterpret_cast<const double2*>(pb[t] + 2 * e)
                                   : make_double2(0, 0);
      rr[t] = mfma(av.x, bv.x, rr[t]);
      ii[t] = mfma(av.y, bv.y, ii[t]);
      ri[t] = mfma(av.x, bv.y, ri[t]);
      ir[t] = mfma(av.y, bv.x, ir[t]);
    }
  }
  // partial[b][chunk][i][j] complex
  double* out = partial + 2 * (((long long)b * nchunks + blockIdx.x) * nba * nbb);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (t < t0 || t >= ntb) continue;
    const int j = t * 16 + (lane & 15);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = ti * 16 + 4 * k + (lane >> 4);
      if (i < nba && j < nbb) {
        out[2 * ((long long)i * nbb + j)] = rr[t][k] + ii[t][k];
        out[2 * ((long long)i * nbb + j) + 1] = ri[t][k] - ir[t][k];
      }
    }
  }
}

// Hermitian Gram, balanced: the workgroup's four waves split the chunk's
// elements into four contiguous runs and every wave computes all upper tile
// pairs (ti <= tj) of its run, so all four SIMDs issue the same MFMA stream
// and each element of A and B is loaded once per workgroup.  The real part
// accumulates Ar'Br + Ai'Bi, the imaginary part Ar'Bi - Ai'Br, chained on two
// accumulators per pair.  The four runs are summed in LDS in a fixed order.
template <int NT>
__global__ void __launch_bounds__(64 * 4)
gram_herm_kernel(const double* A, long long a_bstride, int nba, const double* B,
                 long long b_bstride, int nbb, long long n, long long chunk, const int* active,
                 double* partial) {
  constexpr int NP = NT * (NT + 1) / 2;
  __shared__ double2 red[4][16][17];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int nchunks = gridDim.x;
  const long long c0 = (long long)blockIdx.x * chunk;
  long long c1 = c0 + chunk;
  if (c1 > n) c1 = n;
  // this wave's run: a multiple of 4 elements
  long long q4 = ((c1 - c0 + 15) / 16) * 4;
  long long e0 = c0 + wv * q4;
  long long e1 = e0 + q4;
  if (e1 > c1) e1 = c1;
  if (e0 > c1) e0 = c1;
  const int r = lane & 15, q = lane >> 4;
  const double* pa[NT];
  const double* pb[NT];
  bool aok[NT], bok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int va = t * 16 + r, vb = t * 16 + r;
    aok[t] = va < nba;
    bok[t] = vb < nbb;
    pa[t] = A + 2 * ((long long)b * a_bstride + (long long)(aok[t] ? va : 0) * n);
    pb[t] = B + 2 * ((long long)b * b_bstride + (long long)(bok[t] ? vb : 0) * n);
  }
  d4 re[NP], im[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    re[k] = d4{0, 0, 0, 0};
    im[k] = re[k];
  }
  const long long nks = (e1 - e0 + 3) / 4;
  for (long long st = 0; st < nks; ++st) {
    const long long e = e0 + 4 * st + q;
    const bool eok = e < e1;
    double2 av[NT], bv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      av[t] = (aok[t] && eok) ? *reinterpret_cast<const double2*>(pa[t] + 2 * e)
                              : make_double2(0, 0);
      bv[t] = (bok[t] && eok) ? *reinterpret_cast<const double2*>(pb[t] + 2 * e)
                              : make_double2(0, 0);
    }
    int k = 0;
#pragma unroll
    for (int ti = 0; ti < NT; ++ti) {
#pragma unroll
      for (int tj = ti; tj < NT; ++tj, ++k) {
        re[k] = mfma(av[ti].x, bv[tj].x, re[k]);
        re[k] = mfma(av[ti].y, bv[tj].y, re[k]);
        im[k] = mfma(av[ti].x, bv[tj].y, im[k]);
        im[k] = mfma(-av[ti].y, bv[tj].x, im[k]);
      }
    }
  }
  // partial[b][chunk][i][j]: sum of the four runs, pair by pair
  double* out = partial + 2 * (((long long)b * nchunks + blockIdx.x) * nba * nbb);
  int k = 0;
#pragma unroll
  for (int ti = 0; ti < NT; ++ti) {
#pragma unroll
    for (int tj = ti; tj < NT; ++tj, ++k) {
#pragma unroll
      for (int g = 0; g < 4; ++g) red[wv][4 * g + q][r] = make_double2(re[k][g], im[k][g]);
      __syncthreads();
      {
        const int i = threadIdx.x >> 4, j = threadIdx.x & 15;
        double2 sum = red[0][i][j];
#pragma unroll
        for (int w = 1; w < 4; ++w) {
          sum.x += red[w][i][j].x;
          sum.y += red[w][i][j].y;
        }
        const int gi = ti * 16 + i, gj = tj * 16 + j;
        if (gi < nba && gj < nbb)
          *reinterpret_cast<double2*>(out + 2 * ((long long)gi * nbb + gj)) = sum;
      }
      __syncthreads();
    }
  }
}

// Hermitian Gram A^H B for blocks of nb = 16 T + 8 P vectors (P = 0 or 1), with
// less MFMA work than gram_herm_kernel (which pads nb to whole 16-vector tiles
// and spends four real products on every tile pair):
//  * the last 8 vectors form one packed 16-column operand [re | im], so a pair
//    (full tile, packed tile) costs two MFMAs and (packed, packed) one, their
//    results combined as Re = Ar'Br + Ai'Bi, Im = Ar'Bi - Ai'Br across halves;
//  * with A == B a diagonal tile pair needs Ar'Ar + Ai'Ai for the real part and
//    M = Ar'Ai for the imaginary part, Im = M - M' (three MFMAs instead of four);
//  * the next k-step's elements are loaded while the current one is multiplied.
// For nb = 40 (A == B) a k-step costs 15 MFMAs instead of 24.  Work split and
// the fixed-order reduction of the four waves' runs as in gram_herm_kernel.
template <int T, int P, bool SAME>
__global__ void __launch_bounds__(64 * 4)
gram_hp_kernel(const double* A, long long a_bstride, const double* B, long long b_bstride,
               long long n, long long chunk, const int* active, double* partial) {
  constexpr int nb = 16 * T + 8 * P;
  constexpr int NF = T * (T + 1) / 2;           // full tile pairs, ti <= tj
  // accumulators: full pairs two each (re, im; on the diagonal with A == B: re, M),
  // (full, packed) pairs two each (F1 = Ar'Pb, F2 = Ai'Pb), (packed, packed) one
  constexpr int NACC = 2 * NF + 2 * T * P + P;
  __shared__ double stage[4][2][16][17];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int nchunks = gridDim.x;
  const long long c0 = (long long)blockIdx.x * chunk;
  long long c1 = c0 + chunk;
  if (c1 > n) c1 = n;
  long long q4 = ((c1 - c0 + 15) / 16) * 4;
  long long e0 = c0 + wv * q4;
  long long e1 = e0 + q4;
  if (e1 > c1) e1 = c1;
  if (e0 > c1) e0 = c1;
  const int r = lane & 15, q = lane >> 4;
  const double* pa[T + P];
  const double* pb[T + P];
#pragma unroll
  for (int t = 0; t < T + P; ++t) {
    const int v = t < T ? t * 16 + r : 16 * T + (r & 7);
    pa[t] = A + 2 * ((long long)b * a_bstride + (long long)v * n);
    pb[t] = B + 2 * ((long long)b * b_bstride + (long long)v * n);
  }
  const bool hi = r >= 8;   // packed operand: this lane supplies the imaginary half
  d4 acc[NACC];
#pragma unroll
  for (int k = 0; k < NACC; ++k) acc[k] = d4{0, 0, 0, 0};

  // Two k-steps per loop trip: lane (r, q) loads elements e, e + 1 (e = 8 trip + 2 q)
  // of its vectors with one 32-byte load, so a wave's load instruction covers 8
  // consecutive elements (128 bytes) of each of 16 vectors; k-step u of the trip
  // multiplies element e + u.  The next trip's loads are issued before this
  // trip's MFMAs.
  constexpr int U = 2;
  typedef double dv4 __attribute__((ext_vector_type(4)));
  double2 av[U][T + P], bv[U][T + P];
  // Full trips load without masks and without branches, so that the waits for
  // the next trip's data come only where it is used (a select or a branch right
  // after a load makes the compiler wait for it there); a last, partial trip
  // clamps its addresses into the vector (n >= 2 elements) and zeroes the values
  // past the run's end.
  const long long elast = n >= 2 ? n - 2 : 0;
  auto load = [&](long long trip, bool masked, double2 (&xa)[U][T + P],
                  double2 (&xb)[U][T + P]) {
    const long long e = e0 + 8 * trip + 2 * q;
    const long long ec = masked ? (e < elast ? e : elast) : e;
    const bool ok = !masked || e < e1, ok2 = !masked || e + 1 < e1;
#pragma unroll
    for (int t = 0; t < T + P; ++t) {
      const dv4 va = *reinterpret_cast<const dv4*>(pa[t] + 2 * ec);
      xa[0][t] = make_double2(ok ? va.x : 0.0, ok ? va.y : 0.0);
      xa[1][t] = make_double2(ok2 ? va.z : 0.0, ok2 ? va.w : 0.0);
      if constexpr (!SAME) {
        const dv4 vb = *reinterpret_cast<const dv4*>(pb[t] + 2 * ec);
        xb[0][t] = make_double2(ok ? vb.x : 0.0, ok ? vb.y : 0.0);
        xb[1][t] = make_double2(ok2 ? vb.z : 0.0, ok2 ? vb.w : 0.0);
      } else {
        xb[0][t] = xa[0][t];
        xb[1][t] = xa[1][t];
      }
    }
  };
  auto step = [&](const double2 (&xa)[T + P], const double2 (&xb)[T + P]) {
    const double pbv = P ? (hi ? xb[T + P - 1].y : xb[T + P - 1].x) : 0.0;
    const double pav = P ? (hi ? xa[T + P - 1].y : xa[T + P - 1].x) : 0.0;
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      int k = 0;
#pragma unroll
      for (int ti = 0; ti < T; ++ti) {
#pragma unroll
        for (int tj = ti; tj < T; ++tj, k += 2) {
          if (pass == 0) {
            acc[k] = mfma(xa[ti].x, xb[tj].x, acc[k]);
            acc[k + 1] = mfma(xa[ti].x, xb[tj].y, acc[k + 1]);   // A == B, diagonal: M
          } else {
            acc[k] = mfma(xa[ti].y, xb[tj].y, acc[k]);
            if (!(SAME && ti == tj)) acc[k + 1] = mfma(-xa[ti].y, xb[tj].x, acc[k + 1]);
          }
        }
      }
      if constexpr (P) {
        if (pass == 0) {
#pragma unroll
          for (int ti = 0; ti < T; ++ti, k += 2) {
            acc[k] = mfma(xa[ti].x, pbv, acc[k]);
            acc[k + 1] = mfma(xa[ti].y, pbv, acc[k + 1]);
          }
          acc[k] = mfma(pav, pbv, acc[k]);
        }
      }
    }
  };
  const long long nfull = (e1 - e0) / 8;   // trips of 8 elements inside the run
  auto clampt = [&](long long t) { return t < nfull ? t : (nfull > 0 ? nfull - 1 : 0); };
  // three register sets in rotation: the loads of trip t + 2 are issued while
  // trip t is multiplied (trip indices past the run reload its last trip: the
  // loads need no branch; their products are skipped).  With two blocks (A != B)
  // this leaves one wave per SIMD, still faster than two with one set fewer.
  double2 a1[U][T + P], b1[U][T + P], a2[U][T + P], b2[U][T + P];
  if (nfull > 0) {
    load(0, false, av, bv);
    load(clampt(1), false, a1, b1);
  }
  for (long long tr = 0; tr < nfull; tr += 3) {
    load(clampt(tr + 2), false, a2, b2);
#pragma unroll
    for (int u = 0; u < U; ++u) step(av[u], bv[u]);
    load(clampt(tr + 3), false, av, bv);
    if (tr + 1 < nfull) {
#pragma unroll
      for (int u = 0; u < U; ++u) step(a1[u], b1[u]);
    }
    load(clampt(tr + 4), false, a1, b1);
    if (tr + 2 < nfull) {
#pragma unroll
      for (int u = 0; u < U; ++u) step(a2[u], b2[u]);
    }
  }
  if (e0 + 8 * nfull < e1) {   // the partial last trip
    load(nfull, true, av, bv);
#pragma unroll
    for (int u = 0; u < U; ++u) step(av[u], bv[u]);
  }

  // stage one pair's accumulators (this wave's run), then sum the four runs and
  // write the pair's entries of partial[b][chunk][i][j] (complex)
  double* out = partial + 2 * (((long long)b * nchunks + blockIdx.x) * nb * nb);
  const int ti_ = threadIdx.x >> 4, tj_ = threadIdx.x & 15;   // entry of this thread
  auto put = [&](int m, const d4& v) {
#pragma unroll
    for (int g = 0; g < 4; ++g) stage[wv][m][4 * g + q][r] = v[g];
  };
  auto sum = [&](int m, int i, int j) {
    double s = stage[0][m][i][j];
#pragma unroll
    for (int w = 1; w < 4; ++w) s += stage[w][m][i][j];
    return s;
  };
  auto emit = [&](int gi, int gj, double re, double im) {
    *reinterpret_cast<double2*>(out + 2 * ((long long)gi * nb + gj)) = make_double2(re, im);
  };
  int k = 0;
#pragma unroll
  for (int ti = 0; ti < T; ++ti) {
#pragma unroll
    for (int tj = ti; tj < T; ++tj, k += 2) {
      put(0, acc[k]);
      put(1, acc[k + 1]);
      __syncthreads();
      const double re = sum(0, ti_, tj_);
      const double im = (SAME && ti == tj) ? sum(1, ti_, tj_) - sum(1, tj_, ti_)
                                           : sum(1, ti_, tj_);
      emit(16 * ti + ti_, 16 * tj + tj_, re, im);
      __syncthreads();
    }
  }
  if constexpr (P) {
#pragma unroll
    for (int ti = 0; ti < T; ++ti, k += 2) {
      put(0, acc[k]);
      put(1, acc[k + 1]);
      __syncthreads();
      if (tj_ < 8) {
        const double re = sum(0, ti_, tj_) + sum(1, ti_, tj_ + 8);
        const double im = sum(0, ti_, tj_ + 8) - sum(1, ti_, tj_);
        emit(16 * ti + ti_, 16 * T + tj_, re, im);
      }
      __syncthreads();
    }
    put(0, acc[k]);
    __syncthreads();
    if (ti_ < 8 && tj_ < 8) {
      const double re = sum(0, ti_, tj_) + sum(0, ti_ + 8, tj_ + 8);
      const double im = sum(0, ti_, tj_ + 8) - sum(0, ti_ + 8, tj_);
      emit(16 * T + ti_, 16 * T + tj_, re, im);
    }
  }
}

// General (non-Hermitian) Gram A^H B, balanced as above: the four waves split the
// chunk into four runs and each computes every (A tile, B tile) pair of its run.
// When A is the leading part of B, A's tiles are not loaded a second time.
template <int NTA, int NTB>
__global__ void __launch_bounds__(64 * 4)
gram_gen_kernel(const double* A, long long a_bstride, int nba, const double* B,
                long long b_bstride, int nbb, long long n, long long chunk, const int* active,
                double* partial) {
  // A is the leading part of B (the same vectors): its tiles come from B's loads
  const bool a_is_b = A == B && a_bstride == b_bstride && nba <= nbb && NTA <= NTB;
  __shared__ double2 red[4][16][17];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int nchunks = gridDim.x;
  const long long c0 = (long long)blockIdx.x * chunk;
  long long c1 = c0 + chunk;
  if (c1 > n) c1 = n;
  long long q4 = ((c1 - c0 + 15) / 16) * 4;
  long long e0 = c0 + wv * q4;
  long long e1 = e0 + q4;
  if (e1 > c1) e1 = c1;
  if (e0 > c1) e0 = c1;
  const int r = lane & 15, q = lane >> 4;
  const double* pa[NTA];
  const double* pb[NTB];
  bool aok[NTA], bok[NTB];
#pragma unroll
  for (int t = 0; t < NTA; ++t) {
    const int va = t * 16 + r;
    aok[t] = va < nba;
    pa[t] = A + 2 * ((long long)b * a_bstride + (long long)(aok[t] ? va : 0) * n);
  }
#pragma unroll
  for (int t = 0; t < NTB; ++t) {
    const int vb = t * 16 + r;
    bok[t] = vb < nbb;
    pb[t] = B + 2 * ((long long)b * b_bstride + (long long)(bok[t] ? vb : 0) * n);
  }
  d4 re[NTA * NTB], im[NTA * NTB];
#pragma unroll
  for (int k = 0; k < NTA * NTB; ++k) {
    re[k] = d4{0, 0, 0, 0};
    im[k] = re[k];
  }
  const long long nks = (e1 - e0 + 3) / 4;
  for (long long st = 0; st < nks; ++st) {
    const long long e = e0 + 4 * st + q;
    const bool eok = e < e1;
    double2 av[NTA], bv[NTB];
#pragma unroll
    for (int t = 0; t < NTB; ++t)
      bv[t] = (bok[t] && eok) ? *reinterpret_cast<const double2*>(pb[t] + 2 * e)
                              : make_double2(0, 0);
#pragma unroll
    for (int t = 0; t < NTA; ++t)
      av[t] = a_is_b ? bv[t < NTB ? t : 0]
                     : ((aok[t] && eok) ? *reinterpret_cast<const double2*>(pa[t] + 2 * e)
                                        : make_double2(0, 0));
#pragma unroll
    for (int ti = 0; ti < NTA; ++ti) {
#pragma unroll
      for (int tj = 0; tj < NTB; ++tj) {
        const int k = ti * NTB + tj;
        re[k] = mfma(av[ti].x, bv[tj].x, re[k]);
        re[k] = mfma(av[ti].y, bv[tj].y, re[k]);
        im[k] = mfma(av[ti].x, bv[tj].y, im[k]);
        im[k] = mfma(-av[ti].y, bv[tj].x, im[k]);
      }
    }
  }
  double* out = partial + 2 * (((long long)b * nchunks + blockIdx.x) * nba * nbb);
#pragma unroll
  for (int ti = 0; ti < NTA; ++ti) {
#pragma unroll
    for (int tj = 0; tj < NTB; ++tj) {
      const int k = ti * NTB + tj;
#pragma unroll
      for (int g = 0; g < 4; ++g) red[wv][4 * g + q][r] = make_double2(re[k][g], im[k][g]);
      __syncthreads();
      {
        const int i = threadIdx.x >> 4, j = threadIdx.x & 15;
        double2 sum = red[0][i][j];
#pragma unroll
        for (int w = 1; w < 4; ++w) {
          sum.x += red[w][i][j].x;
          sum.y += red[w][i][j].y;
        }
        const int gi = ti * 16 + i, gj = tj * 16 + j;
        if (gi < nba && gj < nbb)
          *reinterpret_cast<double2*>(out + 2 * ((long long)gi * nbb + gj)) = sum;
      }
      __syncthreads();
    }
  }
}

// fixed-order reduction of the chunk partials: one wave per output entry,
// lane l sums chunks l, l+64, ..., then a shuffle tree (deterministic)
__global__ void __launch_bounds__(256)
gram_reduce_kernel(int nchunks, int nba, int nbb, int hermitian, const int* active,
                   const double* partial, double* out) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int lane = threadIdx.x & 63;
  const int idx = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (idx >= nba * nbb) return;
  const int i = idx / nbb, j = idx % nbb;
  if (hermitian && j < i) return;  // filled from the upper triangle
  const double* p = partial + 2 * ((long long)b * nchunks * nba * nbb + (long long)i * nbb + j);
  const long long cs = 2LL * nba * nbb;
  double re = 0.0, im = 0.0;
  for (int c = lane; c < nchunks; c += 64) {
    re += p[c * cs];
    im += p[c * cs + 1];
  }
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_down(re, off, 64);
    im += __shfl_down(im, off, 64);
  }
  if (lane != 0) return;
  double* o = out + 2 * ((long long)b * nba * nbb);
  if (hermitian) {
    if (i == j) im = 0.0;
    o[2 * ((long long)i * nbb + j)] = re;
    o[2 * ((long long)i * nbb + j) + 1] = im;
    o[2 * ((long long)j * nbb + i)] = re;
    o[2 * ((long long)j * nbb + i) + 1] = -im;
  } else {
    o[2 * ((long long)i * nbb + j)] = re;
    o[2 * ((long long)i * nbb + j) + 1] = im;
  }
}

// ---------------------------------------------------------------------------
// rotate: Y[:, w] = sum_v X[:, v] Q[v][w].  Computed as D^T = Q^T X^T with
// MFMA: M = 16 real output columns (8 output vectors: (w, re), (w, im), ...),
// N = 16 elements, K = 4 real input columns (2 input vectors x (re, im)).
// Each wave owns 16 consecutive elements; it loads all its X values before
// storing, so Y may alias X.  The MFMA A operand depends only on (output
// tile m, k-step s, lane), not on the element tile, so each workgroup first
// lays it out in LDS as qt[m][s][lane] (signs applied, zero outside nin x
// nout); the inner loop is then plain conflict-free LDS reads feeding MFMAs.
// ---------------------------------------------------------------------------
constexpr int kRotWaves = 4;

// The Rayleigh-Ritz form (RITZ): X <- X Q in place and, in the same pass, W Q
// for W = H X (same strides), kept in registers: every output column w gives
//   r2_w += |(W Q)_w - theta_w (X Q)_w|^2       (residual norm, partial sums)
//   Y1_w  = alpha ((W Q)_w - c (X Q)_w)         (the filter's first Chebyshev step)
// and W Q itself is not stored.  Y1 is FP32 (into out32) for members whose
// filter runs in FP32 (f32[b]), else FP64 in place into W.
struct RitzArgs {
  double* W;              // H X, strides of X
  const double* theta;    // [batch][nb] Ritz values (ascending)
  const double* bounds;   // [batch][4]: upper spectral bound first
  const int* f32;         // [batch] FP32 output
  const double* roots;    // product form's roots (null: recurrence)
  float* out32;           // FP32 Y1, strides of W
  double* partial;        // [batch][nb][gridDim.x] residual partial sums
  int nb;
};

template <int NB8, bool RITZ>   // NB8: nin rounded up to a multiple of 8 (zero padding beyond nin, nout)
__global__ void __launch_bounds__(64 * kRotWaves)
rotate_kernel(const double* X, long long x_bstride, double* Y, long long y_bstride, long long n,
              int nin, int nout, const double* Q, const int* active, RitzArgs ra) {
  constexpr int KS = NB8 / 2;            // k-steps of 2 input vectors
  constexpr int MT = NB8 / 8;            // M tiles of 8 output vectors
  extern __shared__ double qt[];         // [MT][KS][64]
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const double* Qb = Q + 2 * ((long long)b * nin * nout);
  for (int t = threadIdx.x; t < MT * KS * 64; t += blockDim.x) {
    const int l = t & 63, s = (t >> 6) % KS, m = (t >> 6) / KS;
    const int rr = l & 15, qq = l >> 4;
    // row mrow of the MFMA result lands in lane group mrow % 4, register
    // mrow / 4; rows are ordered so that every lane ends up holding
    // (w, re), (w, im), (w+1, re), (w+1, im)
    const int w = m * 8 + 2 * (rr & 3) + (rr >> 3);
    const int op = (rr >> 2) & 1;
    const int v = 2 * s + (qq >> 1);
    const int ip = qq & 1;
    double a = 0.0;
    if (v < nin && w < nout) {
      const double qr = Qb[2 * (v * nout + w)], qi = Qb[2 * (v * nout + w) + 1];
      // Yr += Xr Qr - Xi Qi ; Yi += Xr Qi + Xi Qr
      a = op == 0 ? (ip == 0 ? qr : -qi) : (ip == 0 ? qi : qr);
    }
    qt[t] = a;
  }
  // RITZ: residual sums per wave and output vector (lanes 16 q add theirs) and
  // the Ritz values
  __shared__ double red[RITZ ? kRotWaves : 1][RITZ ? NB8 : 1];
  __shared__ double ths[RITZ ? NB8 : 1];
  if constexpr (RITZ) {
    for (int t = threadIdx.x; t < kRotWaves * NB8; t += blockDim.x) (&red[0][0])[t] = 0.0;
    for (int t = threadIdx.x; t < NB8; t += blockDim.x)
      ths[t] = t < ra.nb ? ra.theta[(long long)b * ra.nb + t] : 0.0;
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, q = lane >> 4;
  const int mt = (nout + 7) / 8;
  const double* xb = X + 2 * ((long long)b * x_bstride);
  double* yb = Y + 2 * ((long long)b * y_bstride);
  const long long ntile = (n + 15) / 16;
  // loads need no branch: an element past n reads element n - 1 (its results
  // are not stored) and an input vector past nin reads vector nin - 1 (its
  // operand entries are zero), so all of a tile's loads issue back to back
  int vcl[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int v = 2 * s + (q >> 1);
    vcl[s] = v < nin ? v : nin - 1;
  }
  if constexpr (!RITZ) {
    for (long long tile = (long long)blockIdx.x * kRotWaves + wv; tile < ntile;
         tile += (long long)gridDim.x * kRotWaves) {
      const long long e = tile * 16 + r;
      const bool eok = e < n;
      const long long ec = eok ? e : n - 1;
      // B operand: X^T[k][e], k = 2 v + part
      double xv[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) xv[s] = xb[2 * ((long long)vcl[s] * n + ec) + (q & 1)];
      for (int m = 0; m < mt; ++m) {
        const double* qm = qt + m * KS * 64 + lane;
        d4 acc = d4{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; ++s) acc = mfma(qm[s * 64], xv[s], acc);
        // D[mrow][e]: lane holds (w0, re), (w0, im), (w0+1, re), (w0+1, im)
        const int w0 = m * 8 + 2 * q;
        if (eok) {
          if (w0 < nout)
            *reinterpret_cast<double2*>(yb + 2 * ((long long)w0 * n + e)) = make_double2(acc[0], acc[1]);
          if (w0 + 1 < nout)
            *reinterpret_cast<double2*>(yb + 2 * ((long long)(w0 + 1) * n + e)) = make_double2(acc[2], acc[3]);
        }
      }
    }
  } else {
    // this member's first-step coefficients (the control kernel computes the
    // same ones from the same Ritz values) and output precision; here
    // nout = nin, so every one of the MT output tiles exists
    double r_alpha, r_shift;
    cheb_first_coef(ra.bounds[4 * b], ths[0], ths[ra.nb - 1], ra.roots, &r_alpha, &r_shift);
    const bool r_f32 = ra.f32 && ra.f32[b];
    double* wb = ra.W + 2 * ((long long)b * x_bstride);
    float* o32 = ra.out32 ? ra.out32 + 2 * ((long long)b * x_bstride) : nullptr;
    for (long long tile = (long long)blockIdx.x * kRotWaves + wv; tile < ntile;
         tile += (long long)gridDim.x * kRotWaves) {
      const long long e = tile * 16 + r;
      const bool eok = e < n;
      const long long ec = eok ? e : n - 1;
      double xv[KS], wvv[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) xv[s] = xb[2 * ((long long)vcl[s] * n + ec) + (q & 1)];
#pragma unroll
      for (int s = 0; s < KS; ++s) wvv[s] = wb[2 * ((long long)vcl[s] * n + ec) + (q & 1)];
      for (int m = 0; m < mt; ++m) {
        const double* qm = qt + m * KS * 64 + lane;
        d4 ax = d4{0, 0, 0, 0}, aw = d4{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const double qv = qm[s * 64];
          ax = mfma(qv, xv[s], ax);
          aw = mfma(qv, wvv[s], aw);
        }
        const int w0 = m * 8 + 2 * q;
        double d2[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int w = w0 + j;
          const bool ok = eok && w < nout;
          const double xr = ax[2 * j], xi = ax[2 * j + 1];
          const double ar = aw[2 * j], ai = aw[2 * j + 1], th = ths[w];
          const double dr = ar - th * xr, di = ai - th * xi;
          d2[j] = ok ? fma(dr, dr, di * di) : 0.0;
          const double yr = r_alpha * (ar - r_shift * xr), yi = r_alpha * (ai - r_shift * xi);
          if (ok) {
            const long long o = 2 * ((long long)w * n + e);
            *reinterpret_cast<double2*>(yb + o) = make_double2(xr, xi);
            if (r_f32)
              *reinterpret_cast<float2*>(o32 + o) = make_float2((float)yr, (float)yi);
            else
              *reinterpret_cast<double2*>(wb + o) = make_double2(yr, yi);
          }
        }
        // this tile's sums over the 16 elements of each lane group, added by
        // lane 16 q to the wave's running sums of w0 and w0 + 1
#pragma unroll
        for (int j = 0; j < 2; ++j)
          for (int off = 1; off < 16; off <<= 1) d2[j] += __shfl_xor(d2[j], off, 64);
        if (r == 0) {
          red[wv][w0] += d2[0];
          red[wv][w0 + 1] += d2[1];
        }
      }
    }
    // the waves' sums in a fixed order
    __syncthreads();
    if ((int)threadIdx.x < nout) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < kRotWaves; ++k) t += red[k][threadIdx.x];
      ra.partial[((long long)b * ra.nb + threadIdx.x) * gridDim.x + blockIdx.x] = t;
    }
  }
}

// out[b][j] = sum of the nparts partial sums of (b, j), one workgroup each, in a
// fixed order
__global__ void __launch_bounds__(256)
sum_rows_kernel(int nparts, const double* partial, double* out, const int* active, int per_batch) {
  const int j = blockIdx.x, b = blockIdx.y;
  if (active && !active[b]) return;
  const long long row = (long long)b * per_batch + j;
  double v = 0.0;
  for (int k = threadIdx.x; k < nparts; k += 256) v += partial[row * nparts + k];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) out[row] = red[0] + red[1] + red[2] + red[3];
}

// complex dots conj(a_b) . b_b for one vector per batch member: out[b] = (re, im)
constexpr int kResThreads = 256;

__global__ void __launch_bounds__(kResThreads)
dot_partial_kernel(const double* A, const double* B, long long bstride, long long n,
                   double* partial) {
  const int b = blockIdx.y;
  const double2* a = reinterpret_cast<const double2*>(A) + (long long)b * bstride;
  const double2* c = reinterpret_cast<const double2*>(B) + (long long)b * bstride;
  double sr = 0.0, si = 0.0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const double2 x = a[e], y = c[e];
    sr = fma(x.x, y.x, fma(x.y, y.y, sr));
    si = fma(x.x, y.y, fma(-x.y, y.x, si));
  }
  __shared__ double red[2][kResThreads / 64];
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_down(sr, off, 64);
    si += __shfl_down(si, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = sr;
    red[1][threadIdx.x >> 6] = si;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tr = 0.0, ti = 0.0;
    for (int k = 0; k < kResThreads / 64; ++k) {
      tr += red[0][k];
      ti += red[1][k];
    }
    partial[2 * ((long long)b * gridDim.x + blockIdx.x)] = tr;
    partial[2 * ((long long)b * gridDim.x + blockIdx.x) + 1] = ti;
  }
}

// one wave per batch member: lane l adds partials l, l + 64, ... in turn, then the
// lanes are summed by a fixed shuffle tree (the same order on every run)
__global__ void __launch_bounds__(64)
dot_reduce_kernel(int nparts, const double* partial, double* out) {
  const int b = blockIdx.x;
  const double2* pb = reinterpret_cast<const double2*>(partial) + (long long)b * nparts;
  double sr = 0.0, si = 0.0;
  for (int k = threadIdx.x; k < nparts; k += 64) {
    const double2 v = pb[k];
    sr += v.x;
    si += v.y;
  }
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_down(sr, off, 64);
    si += __shfl_down(si, off, 64);
  }
  if (threadIdx.x == 0) {
    out[2 * b] = sr;
    out[2 * b + 1] = si;
  }
}

// w <- w - alpha v - beta vprev, alpha = Re(dot) and beta = sqrt(norm2prev) read
// from device arrays of (re, im) pairs per batch member
__global__ void lanczos_update_kernel(double* w, const double* v, const double* vprev,
                                      long long n, long long bstride, const double* alpha,
                                      const double* norm2prev) {
  const int b = blockIdx.y;
  const double al = alpha[2 * b], be = norm2prev ? sqrt(norm2prev[2 * b]) : 0.0;
  double2* wb = reinterpret_cast<double2*>(w) + (long long)b * bstride;
  const double2* vb = reinterpret_cast<const double2*>(v) + (long long)b * bstride;
  const double2* pb = vprev ? reinterpret_cast<const double2*>(vprev) + (long long)b * bstride
                            : nullptr;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    double2 x = wb[e];
    const double2 y = vb[e];
    x.x -= al * y.x;
    x.y -= al * y.y;
    if (pb) {
      const double2 z = pb[e];
      x.x -= be * z.x;
      x.y -= be * z.y;
    }
    wb[e] = x;
  }
}

// v <- v / sqrt(norm2[2b])
__global__ void scale_kernel(double* v, long long n, long long bstride, const double* norm2) {
  const int b = blockIdx.y;
  const double nn = norm2[2 * b];
  const double s = nn > 1e-300 ? 1.0 / sqrt(nn) : 0.0;   // breakdown: vector becomes zero
  double2* vb = reinterpret_cast<double2*>(v) + (long long)b * bstride;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    double2 x = vb[e];
    x.x *= s;
    x.y *= s;
    vb[e] = x;
  }
}


template <typename TI, typename TO>
__global__ void cast_kernel(const TI* in, TO* out, long long count) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (long long)gridDim.x * blockDim.x)
    out[e] = (TO)in[e];
}

// counter-based generator: splitmix64 of (seed, batch, vector, element)
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

__global__ void random_kernel(double* X, long long n, int nvec, long long bstride,
                              unsigned long long seed) {
  const int b = blockIdx.z, v = blockIdx.y;
  double* xb = X + 2 * ((long long)b * bstride + (long long)v * n);
  const unsigned long long base =
      splitmix64(seed ^ splitmix64(((unsigned long long)b << 32) | (unsigned)v));
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const unsigned long long r = splitmix64(base + (unsigned long long)e);
    const double re = ((double)(r >> 11) * 0x1.0p-53) * 2.0 - 1.0;
    const unsigned long long r2 = splitmix64(r);
    const double im = ((double)(r2 >> 11) * 0x1.0p-53) * 2.0 - 1.0;
    xb[2 * e] = re;
    xb[2 * e + 1] = im;
  }
}

unsigned grid_for(long long count, int threads, unsigned cap = 4096) {
  long long g = (count + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

int gram_chunks(long long n, int batch) {
  // aim for about 2048 workgroups (x row-tile blocks) over the batch
  long long per = 2048 / (batch > 0 ? batch : 1);
  if (per < 8) per = 8;
  long long maxc = (n + kGramChunkMin - 1) / kGramChunkMin;
  if (per > maxc) per = maxc;
  if (per < 1) per = 1;
  return (int)per;
}

size_t gram_partial_bytes(int nb, long long n, int batch) {
  return (size_t)gram_chunks(n, batch) * batch * nb * nb * 16;
}

hipError_t launch_gram(const BlockDesc& A, const BlockDesc& B, int hermitian, int batch,
                       double* partial, double* out, const int* active, hipStream_t s) {
  const long long n = A.n;
  const int nchunks = gram_chunks(n, batch);
  long long chunk = (n + nchunks - 1) / nchunks;
  chunk = (chunk + 15) & ~15LL;
  const int nta = (A.nvec + 15) / 16, ntb = (B.nvec + 15) / 16;
  const bool same = A.ptr == B.ptr && A.bstride == B.bstride;
  if (hermitian && A.nvec == B.nvec && A.nvec % 8 == 0 && A.nvec >= 16 && A.nvec <= 64) {
    dim3 grid((unsigned)nchunks, (unsigned)batch);
#define HKP_HP(T, P)                                                                          \
  (same ? gram_hp_kernel<T, P, true><<<grid, 256, 0, s>>>(A.ptr, A.bstride, B.ptr, B.bstride,  \
                                                          n, chunk, active, partial)          \
        : gram_hp_kernel<T, P, false><<<grid, 256, 0, s>>>(A.ptr, A.bstride, B.ptr,           \
                                                           B.bstride, n, chunk, active,        \
                                                           partial))
    switch (A.nvec / 8) {
      case 2: HKP_HP(1, 0); break;
      case 3: HKP_HP(1, 1); break;
      case 4: HKP_HP(2, 0); break;
      case 5: HKP_HP(2, 1); break;
      case 6: HKP_HP(3, 0); break;
      case 7: HKP_HP(3, 1); break;
      default: HKP_HP(4, 0); break;
    }
#undef HKP_HP
  } else if (hermitian && A.nvec == B.nvec) {
    dim3 grid((unsigned)nchunks, (unsigned)batch);
    switch (nta) {
      case 1: gram_herm_kernel<1><<<grid, 256, 0, s>>>(A.ptr, A.bstride, A.nvec, B.ptr, B.bstride, B.nvec, n, chunk, active, partial); break;
      case 2: gram_herm_kernel<2><<<grid, 256, 0, s>>>(A.ptr, A.bstride, A.nvec, B.ptr, B.bstride, B.nvec, n, chunk, active, partial); break;
      case 3: gram_herm_kernel<3><<<grid, 256, 0, s>>>(A.ptr, A.bstride, A.nvec, B.ptr, B.bstride, B.nvec, n, chunk, active, partial); break;
      case 4: gram_herm_kernel<4><<<grid, 256, 0, s>>>(A.ptr, A.bstride, A.nvec, B.ptr, B.bstride, B.nvec, n, chunk, active, partial); break;
      default: return hipErrorInvalidValue;
    }
  } else if (!hermitian) {
    dim3 grid((unsigned)nchunks, (unsigned)batch);
#define HKP_GEN(TA, TB)                                                                       \
  gram_gen_kernel<TA, TB><<<grid, 256, 0, s>>>(A.ptr, A.bstride, A.nvec, B.ptr, B.bstride,    \
                                               B.nvec, n, chunk, active, partial)
    if (nta < 1 || nta > 4 || ntb < 1 || ntb > 4) return hipErrorInvalidValue;
    switch (4 * (nta - 1) + (ntb - 1)) {
      case 0: HKP_GEN(1, 1); break;
      case 1: HKP_GEN(1, 2); break;
      case 2: HKP_GEN(1, 3); break;
      case 3: HKP_GEN(1, 4); break;
      case 4: HKP_GEN(2, 1); break;
      case 5: HKP_GEN(2, 2); break;
      case 6: HKP_GEN(2, 3); break;
      case 7: HKP_GEN(2, 4); break;
      case 8: HKP_GEN(3, 1); break;
      case 9: HKP_GEN(3, 2); break;
      case 10: HKP_GEN(3, 3); break;
      case 11: HKP_GEN(3, 4); break;
      case 12: HKP_GEN(4, 1); break;
      case 13: HKP_GEN(4, 2); break;
      case 14: HKP_GEN(4, 3); break;
      default: HKP_GEN(4, 4); break;
    }
#undef HKP_GEN
  } else {
    dim3 grid((unsigned)nchunks, (unsigned)((nta + 3) / 4), (unsigned)batch);
    switch (ntb) {
      case 1: gram_partial_kernel<1><<<grid, 256, 0, s>>>(A.ptr, A.bstride, A.nvec, B.ptr, B.bstride, B.nvec, n, chunk, hermitian, active, partial); break;
      case 2: gram_partial_kernel<2><<<grid, 256, 0, s>>>(A.ptr, A.bstride, A.nvec, B.ptr, B.bstride, B.nvec, n, chunk, hermitian, active, partial); break;
      case 3: gram_partial_kernel<3><<<grid, 256, 0, s>>>(A.ptr, A.bstride, A.nvec, B.ptr, B.bstride, B.nvec, n, chunk, hermitian, active, partial); break;
      case 4: gram_partial_kernel<4><<<grid, 256, 0, s>>>(A.ptr, A.bstride, A.nvec, B.ptr, B.bstride, B.nvec, n, chunk, hermitian, active, partial); break;
      default: return hipErrorInvalidValue;
    }
  }
  const int cnt = A.nvec * B.nvec;
  dim3 g2((unsigned)((cnt + 3) / 4), (unsigned)batch);
  gram_reduce_kernel<<<g2, 256, 0, s>>>(nchunks, A.nvec, B.nvec, hermitian, active, partial, out);
  return hipGetLastError();
}

int rotate_blocks(long long n, int batch) {
  const long long ntile = (n + 15) / 16;
  long long g = (ntile + kRotWaves - 1) / kRotWaves;
  const long long cap = 4096 / (batch > 0 ? batch : 1) + 1;
  if (g > cap) g = cap;
  return (int)(g < 1 ? 1 : g);
}

namespace {
template <bool RITZ>
hipError_t rotate_any(const BlockDesc& X, const BlockDesc& Y, int nin, int nout,
                      const double* Q, int batch, const int* active, const RitzArgs& ra,
                      hipStream_t s) {
  if (nin > HKP_NB_MAX || nout > nin) return hipErrorInvalidValue;
  dim3 grid((unsigned)rotate_blocks(X.n, batch), (unsigned)batch);
  // operand table [NB8/8][NB8/2][64] doubles, NB8 = nin rounded up to 8
  const int nb8 = (nin + 7) / 8 * 8;
  const size_t lds = (size_t)(nb8 / 8) * (nb8 / 2) * 64 * 8;
#define HKP_ROT(NB8) rotate_kernel<NB8, RITZ><<<grid, 64 * kRotWaves, lds, s>>>(X.ptr, X.bstride, Y.ptr, Y.bstride, X.n, nin, nout, Q, active, ra)
  switch (nb8) {
    case 8: HKP_ROT(8); break;
    case 16: HKP_ROT(16); break;
    case 24: HKP_ROT(24); break;
    case 32: HKP_ROT(32); break;
    case 40: HKP_ROT(40); break;
    case 48: HKP_ROT(48); break;
    case 56: HKP_ROT(56); break;
    case 64: HKP_ROT(64); break;
    default: return hipErrorInvalidValue;
  }
#undef HKP_ROT
  return hipGetLastError();
}
}  // namespace

hipError_t launch_rotate(const BlockDesc& X, const BlockDesc& Y, int nin, int nout,
                         const double* Q, int batch, const int* active, hipStream_t s) {
  return rotate_any<false>(X, Y, nin, nout, Q, batch, active, RitzArgs{}, s);
}

hipError_t launch_ritz(const BlockDesc& X, const BlockDesc& W, int nb, const double* Q,
                       const double* theta, const double* bounds, const double* roots,
                       const int* f32, float* out32, int batch, double* partial, double* r2,
                       const int* active, hipStream_t s) {
  if (W.bstride != X.bstride || W.n != X.n || W.nvec < nb || X.nvec < nb)
    return hipErrorInvalidValue;
  const RitzArgs ra{W.ptr, theta, bounds, f32, roots, out32, partial, nb};
  hipError_t e = rotate_any<true>(X, X, nb, nb, Q, batch, active, ra, s);
  if (e != hipSuccess) return e;
  sum_rows_kernel<<<dim3((unsigned)nb, (unsigned)batch), 256, 0, s>>>(
      rotate_blocks(X.n, batch), partial, r2, active, nb);
  return hipGetLastError();
}


hipError_t launch_cast(const void* in, int in_fp64, void* out, int out_fp64, long long count,
                       hipStream_t s) {
  const unsigned g = grid_for(count, 256, 16384);
  if (in_fp64 && !out_fp64)
    cast_kernel<double, float><<<g, 256, 0, s>>>((const double*)in, (float*)out, count);
  else if (!in_fp64 && out_fp64)
    cast_kernel<float, double><<<g, 256, 0, s>>>((const float*)in, (double*)out, count);
  else if (in_fp64)
    cast_kernel<double, double><<<g, 256, 0, s>>>((const double*)in, (double*)out, count);
  else
    cast_kernel<float, float><<<g, 256, 0, s>>>((const float*)in, (float*)out, count);
  return hipGetLastError();
}

hipError_t launch_random_block(double* X, long long n, int nvec, int batch, long long bstride,
                               unsigned long long seed, hipStream_t s) {
  dim3 grid(grid_for(n, 256, 1024), (unsigned)nvec, (unsigned)batch);
  random_kernel<<<grid, 256, 0, s>>>(X, n, nvec, bstride, seed);
  return hipGetLastError();
}

int dot_parts() { return 256; }

hipError_t launch_dots(const double* a, const double* b, long long n, int batch,
                       long long bstride, double* partial, double* out, hipStream_t s) {
  const int parts = dot_parts();
  dim3 grid((unsigned)parts, (unsigned)batch);
  dot_partial_kernel<<<grid, kResThreads, 0, s>>>(a, b, bstride, n, partial);
  dot_reduce_kernel<<<batch, 64, 0, s>>>(parts, partial, out);
  return hipGetLastError();
}

hipError_t launch_lanczos_update(double* w, const double* v, const double* vprev, long long n,
                                 int batch, long long bstride, const double* alpha,
                                 const double* beta, hipStream_t s) {
  dim3 grid(grid_for(n, 256, 2048), (unsigned)batch);
  lanczos_update_kernel<<<grid, 256, 0, s>>>(w, v, vprev, n, bstride, alpha, beta);
  return hipGetLastError();
}

hipError_t launch_scale(double* v, long long n, int batch, long long bstride,
                        const double* norm2, hipStream_t s) {
  dim3 grid(grid_for(n, 256, 2048), (unsigned)batch);
  scale_kernel<<<grid, 256, 0, s>>>(v, n, bstride, norm2);
  return hipGetLastError();
}

}  // namespace hkp
