// Host orchestration of the Chebyshev-filtered subspace iteration (the
// Rayleigh-Chebyshev method named in the paper, Sec. II.B):
//
//   bounds   k-step Lanczos -> upper spectral bound b
//   init     random block, SVQB, Rayleigh-Ritz
//   repeat   filter:  Y = p_m(H) X, scaled three-term Chebyshev recurrence on
//                     [a_cut, b] (a_cut = largest Ritz value of the block,
//                     normalised at the lowest Ritz value) -- m fused stencil
//                     steps, FP64 or FP32 (mixed precision)
//            orth:    SVQB twice (Gram, Jacobi eig, rotate), FP64
//            RR:      W = H X (FP64), X^H W, Jacobi eig; one pass over X and W
//                     gives X <- X Q, ||(W Q)_j - theta_j (X Q)_j|| and the next
//                     filter's first step alpha (W Q - c X Q) (W Q is not stored)
//            control: convergence, locking, precision and the next interval
//   until    the nev lowest residuals are <= tol
//
// All per-iteration decisions (convergence, precision switch, filter
// coefficients) are made on the device, so one outer iteration is a fixed
// sequence of launches.  Eager mode reads the flags after every iteration;
// graph mode records a batch of iterations once and replays it.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include "hkp_internal.h"
#include "solver.h"

namespace hkp {

namespace {

#define HKP_CHECK(x)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      throw HipError(std::string(#x) + ": " + hipGetErrorString(e_));                  \
  } while (0)

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int kLanczosSteps = 40;
constexpr int kKmax = 200;       // largest Chebyshev degree
constexpr int kDotParts = 256;

struct Layout {
  size_t D64, D32, w64, v64, w32, v32, X, W, A32, B32, C32, E32, gram, mat1, mat2, mat3, mat4,
      theta, lam,
      r2, rpart, coef, bounds, flags, active, act32, act64, lock, sw, work, again, status, lal,
      lnrm,
      lpart, zero, roots, total;
};

Layout make_layout(const Plan& p) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes);
    return o;
  };
  const size_t B = p.batch;
  const size_t N = p.N, n6 = p.n6;
  L.D64 = take(B * 6 * N * 8);
  L.D32 = p.mixed ? take(B * 6 * N * 4) : 0;
  L.w64 = take((size_t)p.nz * 16);
  L.v64 = take((size_t)p.nz * p.nx * 16);
  L.w32 = take((size_t)p.nz * 8);
  L.v32 = take((size_t)p.nz * p.nx * 8);
  L.X = take(B * p.nb * n6 * 16);
  L.W = take(B * p.nb * n6 * 16);
  if (p.mixed) {
    L.A32 = take(B * p.nb * n6 * 8);
    L.B32 = take(B * p.nb * n6 * 8);
    if (p.two_step) {   // the two outputs of a two-step pass
      L.C32 = take(B * p.nb * n6 * 8);
      L.E32 = take(B * p.nb * n6 * 8);
    }
  }
  L.gram = take(gram_partial_bytes(p.nb, n6, p.batch));
  L.mat1 = take(B * p.nb * p.nb * 16);
  L.mat2 = take(B * p.nb * p.nb * 16);
  L.mat3 = take(B * p.nb * p.nb * 16);
  L.mat4 = take(B * p.nb * p.nb * 16);
  L.theta = take(B * p.nb * 8);
  L.lam = take(B * p.nb * 8);
  L.r2 = take(B * p.nb * 8);
  L.rpart = take(B * p.nb * (size_t)rotate_blocks(p.n6, p.batch) * 8);   // residual partials
  L.coef = take(B * kKmax * 4 * 8);
  L.bounds = take(B * 4 * 8);
  L.flags = take(B * 8 * 4);
  L.active = take(B * 4);
  L.act32 = take(B * 4);
  L.act64 = take(B * 4);
  L.lock = take(B * 4);
  L.sw = take(B * 4);
  L.work = take(3 * (B + 1) * 4);
  L.again = take(B * 4);
  L.status = take(B * 4 + 4);
  L.lal = take((size_t)kLanczosSteps * B * 16);
  L.lnrm = take((size_t)(kLanczosSteps + 1) * B * 16);
  L.lpart = take(B * kDotParts * 16);
  L.zero = take(256);   // zeros (the hard wall's values for the two-step copies)
  L.roots = take(kKmax * 8);   // the product form's roots on [-1, 1], Leja order
  L.total = off;
  return L;
}

// largest and smallest eigenvalue of a symmetric tridiagonal matrix (Sturm bisection)
int sturm_count(const std::vector<double>& a, const std::vector<double>& b2, double x) {
  // number of eigenvalues < x; b2[i] = beta_i^2 couples i-1 and i
  int cnt = 0;
  double d = a[0] - x;
  if (d < 0) ++cnt;
  for (size_t i = 1; i < a.size(); ++i) {
    if (d == 0) d = 1e-300;
    d = a[i] - x - b2[i] / d;
    if (d < 0) ++cnt;
  }
  return cnt;
}

void tridiag_extremes(const std::vector<double>& a, const std::vector<double>& b2, double* lo,
                      double* hi) {
  const size_t k = a.size();
  double gl = a[0], gh = a[0];
  for (size_t i = 0; i < k; ++i) {
    double r = 0;
    if (i > 0) r += std::sqrt(b2[i]);
    if (i + 1 < k) r += std::sqrt(b2[i + 1]);
    gl = std::min(gl, a[i] - r);
    gh = std::max(gh, a[i] + r);
  }
  const int kk = (int)k;
  double l = gl, h = gh;
  for (int it = 0; it < 200; ++it) {   // largest: count(x) < k
    const double m = 0.5 * (l + h);
    if (sturm_count(a, b2, m) < kk) l = m; else h = m;
  }
  *hi = h;
  l = gl;
  h = gh;
  for (int it = 0; it < 200; ++it) {   // smallest: count(x) >= 1
    const double m = 0.5 * (l + h);
    if (sturm_count(a, b2, m) >= 1) h = m; else l = m;
  }
  *lo = l;
}

// per-launch accounting of the stencil kernel: algorithmic bytes always,
// event-timed durations when requested (eager mode)
struct StencilStats {
  bool timed = false;
  std::vector<hipEvent_t> ev;   // start/stop pairs
  std::vector<int> kind;        // 0: FP32 stencil, 1: FP64
  std::vector<double> bytes;
  size_t used = 0;
  double hx_bytes = 0, t32 = 0, t64 = 0, b32 = 0, b64 = 0, t32x2 = 0, b32x2 = 0;
  long long n32 = 0, n64 = 0, n32x2 = 0;
  ~StencilStats() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
  // nvec_done: vectors the launch processes summed over the active members
  // (< 0: every vector of every active member)
  void launch(const StencilLaunch& a, const StencilConsts<double>& c, hipStream_t s,
              long long N, int active_members, double nvec_done = -1) {
    const double sin = a.fp64 ? 16 : 8;
    const double sold = a.old ? (a.old_fp64 ? 16 : 8) : 0;
    const double sout = a.out_fp64 ? 16 : 8;
    if (nvec_done < 0) nvec_done = (double)active_members * a.nvec;
    const double b = (double)N * a.ncomp * nvec_done * (sin + sold + sout) +
                     (double)active_members * N * (a.strain ? 6 : 1) * (a.fp64 ? 8 : 4);
    hx_bytes += b;
    if (!timed) {
      HKP_CHECK(launch_stencil(a, c, s));
      return;
    }
    if (2 * used + 2 > ev.size()) {
      hipEvent_t e0, e1;
      HKP_CHECK(hipEventCreate(&e0));
      HKP_CHECK(hipEventCreate(&e1));
      ev.push_back(e0);
      ev.push_back(e1);
      kind.push_back(0);
      bytes.push_back(0);
    }
    HKP_CHECK(hipEventRecord(ev[2 * used], s));
    HKP_CHECK(launch_stencil(a, c, s));
    HKP_CHECK(hipEventRecord(ev[2 * used + 1], s));
    kind[used] = a.fp64 ? 1 : 0;
    bytes[used] = b;
    ++used;
  }
  // a two-step pass: algorithmic bytes of the two recurrence steps it performs
  // (each step: its blocks read and written plus the fields, as a one-step pass)
  void launch2(const Stencil2Launch& a, const StencilConsts<double>& c, hipStream_t s,
               long long N, int active_members, double nvec_done = -1) {
    if (nvec_done < 0) nvec_done = (double)active_members * a.nvec;
    const double b = 2.0 * ((double)N * 6 * nvec_done * 3 * 8 +
                            (double)active_members * N * (a.strain ? 6 : 1) * 4);
    hx_bytes += b;
    if (!timed) {
      HKP_CHECK(launch_stencil2(a, c, s));
      return;
    }
    if (2 * used + 2 > ev.size()) {
      hipEvent_t e0, e1;
      HKP_CHECK(hipEventCreate(&e0));
      HKP_CHECK(hipEventCreate(&e1));
      ev.push_back(e0);
      ev.push_back(e1);
      kind.push_back(0);
      bytes.push_back(0);
    }
    HKP_CHECK(hipEventRecord(ev[2 * used], s));
    HKP_CHECK(launch_stencil2(a, c, s));
    HKP_CHECK(hipEventRecord(ev[2 * used + 1], s));
    kind[used] = 2;
    bytes[used] = b;
    ++used;
  }
  void collect() {
    if (!timed || used == 0) return;
    HKP_CHECK(hipEventSynchronize(ev[2 * used - 1]));
    for (size_t i = 0; i < used; ++i) {
      float ms = 0;
      HKP_CHECK(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
      if (kind[i] == 2) {
        t32x2 += ms * 1e-3;
        b32x2 += bytes[i];
        ++n32x2;
      } else if (kind[i]) {
        t64 += ms * 1e-3;
        b64 += bytes[i];
        ++n64;
      } else {
        t32 += ms * 1e-3;
        b32 += bytes[i];
        ++n32;
      }
    }
    used = 0;
  }
};

struct Ctx {
  StencilStats* ss = nullptr;
  int active_members = 1;   // host view of unconverged Hamiltonians (byte accounting)
  double filtered_vectors = -1;   // host view of the vectors the filter processes (-1: all)
  Plan p;
  Layout L;
  char* ws;
  hipStream_t s;
  StencilConsts<double> consts;
  bool field;
  bool field_z;   // Bz != 0: y-link phases vary along x
  bool strain;
  template <typename T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  long long bstride() const { return (long long)p.nb * p.n6; }
  BlockDesc blk(size_t off, int nvec) const {
    return BlockDesc{at<double>(off), p.n6, nvec, bstride()};
  }
  // work table of the FP32 filter (0), FP64 filter (1) or whole block (2)
  const int* work(int k) const { return at<int>(L.work) + k * (p.batch + 1); }
  Control control() const {
    return Control{at<double>(L.theta), at<double>(L.r2),     at<double>(L.coef),
                   at<double>(L.bounds), at<int>(L.flags),    at<int>(L.active),
                   at<int>(L.act32),     at<int>(L.act64),    at<int>(L.lock),
                   at<int>(L.sw),        p.product ? at<double>(L.roots) : nullptr,
                   at<int>(L.work)};
  }
};

StencilLaunch base_launch(const Ctx& c, bool fp64, int nvec) {
  StencilLaunch a{};
  a.nx = c.p.nx;
  a.ny = c.p.ny;
  a.nz = c.p.nz;
  a.nvec = nvec;
  a.batch = c.p.batch;
  a.D = fp64 ? (const void*)c.at<double>(c.L.D64) : (const void*)c.at<float>(c.L.D32);
  a.D_bstride = 6LL * c.p.N;
  a.strain = c.strain;
  if (c.field) {
    a.wtab = fp64 ? (const void*)c.at<double>(c.L.w64) : (const void*)c.at<float>(c.L.w32);
    a.vtab = fp64 ? (const void*)c.at<double>(c.L.v64) : (const void*)c.at<float>(c.L.v32);
    a.phase_general = c.field_z;
  }
  a.tile_y = c.p.st.tile_y;
  a.vgroup = c.p.st.vgroup;
  a.dma = c.p.st.dma;
  a.zsplit = c.p.st.zsplit;
  a.fp64 = fp64;
  a.ncomp = c.p.ncomp;
  a.coef.coef = nullptr;
  a.coef.alpha = 1.0;
  a.coef.shift = 0.0;
  a.coef.beta = 0.0;
  return a;
}

// W = H X over the whole block (FP64)
void apply_block(const Ctx& c, size_t x_off, size_t w_off, const int* active) {
  StencilLaunch a = base_launch(c, true, c.p.nb);
  a.in = c.at<double>(x_off);
  a.in_bstride = c.bstride();
  a.out = c.at<double>(w_off);
  a.out_fp64 = 1;
  a.out_bstride = c.bstride();
  a.active = active;
  a.work = c.work(2);
  c.ss->launch(a, c.consts, c.s, c.p.N, c.active_members);
}

// The roots of the degree-m Chebyshev polynomial on [-1, 1], cos((2i - 1) pi / 2m),
// in Leja order: the largest first, then each maximising the product of its
// distances to those before it (log sums; ties to the lower index).  Applied in
// this order the scaled factors (H - r) / (a0 - r) keep every partial product
// small on the damped interval, so the product form runs in FP32 as the
// recurrence does.  The order is invariant under the affine map onto [a_cut, b].
RootTable leja_cheb_roots(int m) {
  RootTable t{};
  std::vector<double> x(m), logp(m, 0.0);
  std::vector<char> used(m, 0);
  for (int i = 0; i < m; ++i) x[i] = std::cos((2.0 * i + 1.0) * M_PI / (2.0 * m));
  for (int k = 0; k < m; ++k) {
    int best = -1;
    for (int i = 0; i < m; ++i) {
      if (used[i]) continue;
      const double score = k == 0 ? std::fabs(x[i]) : logp[i];
      const double bs = best < 0 ? 0.0 : (k == 0 ? std::fabs(x[best]) : logp[best]);
      if (best < 0 || score > bs) best = i;
    }
    used[best] = 1;
    t.x[k] = x[best];
    for (int i = 0; i < m; ++i)
      if (!used[i]) logp[i] += std::log(std::fabs(x[i] - x[best]));
  }
  return t;
}

// Chebyshev filter of degree m (even) in FP64: the filtered block ends in X.
// The first step Y1 = alpha (H - c) X is already in W (written by the
// Rayleigh-Ritz step), except for members that have just left the FP32 filter
// (their Y1 went to the FP32 buffer): for those one stencil pass computes it.
void filter64(const Ctx& c, const int* active, int m) {
  const int kstride = kKmax * 4;
  if (c.p.mixed) {
    StencilLaunch a = base_launch(c, true, c.p.nb);
    a.in = c.at<double>(c.L.X);
    a.in_bstride = c.bstride();
    a.out = c.at<double>(c.L.W);
    a.out_fp64 = 1;
    a.out_bstride = c.bstride();
    a.coef.coef = c.at<double>(c.L.coef);
    a.coef.stride = kstride;
    a.active = c.at<int>(c.L.sw);
    a.lock = c.at<int>(c.L.lock);
    HKP_CHECK(launch_stencil(a, c.consts, c.s));
  }
  size_t cur = c.L.W, oth = c.L.X;
  for (int k = 1; k < m; ++k) {
    StencilLaunch a = base_launch(c, true, c.p.nb);
    a.in = c.at<double>(cur);
    a.in_bstride = c.bstride();
    a.old = c.p.product ? nullptr : c.at<double>(oth);
    a.old_fp64 = 1;
    a.old_bstride = c.bstride();
    a.out = c.at<double>(oth);
    a.out_fp64 = 1;
    a.out_bstride = c.bstride();
    a.coef.coef = c.at<double>(c.L.coef) + 4 * k;
    a.coef.stride = kstride;
    a.active = active;
    a.lock = c.at<int>(c.L.lock);
    a.work = c.work(1);
    c.ss->launch(a, c.consts, c.s, c.p.N, c.active_members, c.filtered_vectors);
    std::swap(cur, oth);
  }
}

// Chebyshev filter in FP32 (mixed precision): the first step Y1 (FP32, written
// by the Rayleigh-Ritz step) and X (FP64) start it, the last step writes FP64
// into X
void filter32(const Ctx& c, const int* active, int m) {
  const int kstride = kKmax * 4;
  float* A = c.at<float>(c.L.A32);
  float* Bf = c.at<float>(c.L.B32);
  // two-step passes for the middle of the recurrence when tuned for this grid
  Stencil2Launch t2{};
  bool two = false;
  if (c.p.two_step && c.p.st.t2x > 0) {
    t2.nx = c.p.nx;
    t2.ny = c.p.ny;
    t2.nz = c.p.nz;
    t2.nvec = c.p.nb;
    t2.batch = c.p.batch;
    t2.bstride = c.bstride();
    t2.D = c.at<float>(c.L.D32);
    t2.D_bstride = 6LL * c.p.N;
    t2.strain = c.strain;
    if (c.field) {
      t2.wtab = c.at<float>(c.L.w32);
      t2.vtab = c.at<float>(c.L.v32);
      t2.phase_general = c.field_z;
    }
    t2.coef_stride = kstride;
    t2.zero = c.at<float>(c.L.zero);
    t2.active = active;
    t2.lock = c.at<int>(c.L.lock);
    t2.work = c.work(0);
    t2.tile_x = c.p.st.t2x;
    t2.tile_y = c.p.st.t2y;
    t2.vgroup = c.p.st.vgroup;
    two = stencil2_supported(t2);
  }
  if (c.p.product) {
    // product form: step k maps Y_k to Y_{k+1} (FP32 buffers in turn), the last
    // step writes FP64 into X
    float* buf[2] = {A, Bf};
    int cur = 0;
    for (int k = 1; k < m; ++k) {
      const bool last = k == m - 1;
      StencilLaunch a = base_launch(c, false, c.p.nb);
      a.in = buf[cur];
      a.in_bstride = c.bstride();
      a.out = last ? (void*)c.at<double>(c.L.X) : (void*)buf[1 - cur];
      a.out_fp64 = last ? 1 : 0;
      a.out_bstride = c.bstride();
      a.coef.coef = c.at<double>(c.L.coef) + 4 * k;
      a.coef.stride = kstride;
      a.active = active;
      a.lock = c.at<int>(c.L.lock);
      a.work = c.work(0);
      c.ss->launch(a, c.consts, c.s, c.p.N, c.active_members, c.filtered_vectors);
      cur = 1 - cur;
    }
    return;
  }
  float* spare[2] = {two ? c.at<float>(c.L.C32) : nullptr, two ? c.at<float>(c.L.E32) : nullptr};
  // step k: in = Y_k (FP32), old = Y_{k-1} (X in FP64 for k = 1), out = Y_{k+1}
  const void* in = A;
  const void* old = c.at<double>(c.L.X);
  int old64 = 1;
  float* free32 = Bf;
  auto one_step = [&](int k) {
    const bool last = k == m - 1;
    StencilLaunch a = base_launch(c, false, c.p.nb);
    a.in = in;
    a.in_bstride = c.bstride();
    a.old = old;
    a.old_fp64 = old64;
    a.old_bstride = c.bstride();
    void* out = last ? (void*)c.at<double>(c.L.X) : (void*)(old64 ? free32 : (float*)old);
    a.out = out;
    a.out_fp64 = last ? 1 : 0;
    a.out_bstride = c.bstride();
    a.coef.coef = c.at<double>(c.L.coef) + 4 * k;
    a.coef.stride = kstride;
    a.active = active;
    a.lock = c.at<int>(c.L.lock);
    a.work = c.work(0);
    c.ss->launch(a, c.consts, c.s, c.p.N, c.active_members, c.filtered_vectors);
    old = in;
    old64 = 0;
    in = out;
  };
  int k = 1;
  if (k < m) one_step(k++);   // reads X (FP64) as Y_0
  if (two) {
    // steps 2 .. m-2 in pairs (one step first when their count is odd); a pair
    // writes the two FP32 blocks it does not read
    if (((m - 3) & 1) && k < m - 1) one_step(k++);
    while (k + 1 < m - 1) {
      t2.in = in;
      t2.old = old;
      t2.out1 = spare[0];
      t2.out2 = spare[1];
      t2.coef1 = c.at<double>(c.L.coef) + 4 * k;
      t2.coef2 = c.at<double>(c.L.coef) + 4 * (k + 1);
      c.ss->launch2(t2, c.consts, c.s, c.p.N, c.active_members, c.filtered_vectors);
      float* was_in = (float*)in;
      float* was_old = (float*)old;
      old = spare[0];
      in = spare[1];
      spare[0] = was_in;
      spare[1] = was_old;
      k += 2;
    }
  }
  while (k < m) one_step(k++);
}

// SVQB factor of X: S = D U diag(lambda)^-1/2 from X^H X (X S orthonormal) into
// `out`; `again` (optional) receives the per-member need for a second pass
void svqb_factor(const Ctx& c, const int* active, size_t out, int* again = nullptr) {
  BlockDesc X = c.blk(c.L.X, c.p.nb);
  HKP_CHECK(launch_gram(X, X, 1, c.p.batch, c.at<double>(c.L.gram), c.at<double>(c.L.mat1),
                        active, c.s));
  HKP_CHECK(launch_heev(c.at<double>(c.L.mat1), c.p.nb, c.p.batch, (long long)c.p.nb * c.p.nb,
                        c.at<double>(c.L.lam), c.at<double>(out), 1, c.at<int>(c.L.status),
                        active, c.s, again));
}

// orthonormalise X by SVQB: its factor S goes to mat3 and is applied by the
// Rayleigh-Ritz rotation (X S Q in one pass over the block).  Members whose Gram
// matrix was ill conditioned (one pass would leave an orthogonality error
// ~ eps kappa) are rotated now and take a second pass; their mat3 is I.
void orthonormalise(const Ctx& c, const int* active) {
  int* again = c.at<int>(c.L.again);
  const long long ms = (long long)c.p.nb * c.p.nb;
  BlockDesc X = c.blk(c.L.X, c.p.nb);
  svqb_factor(c, active, c.L.mat3, again);
  HKP_CHECK(launch_rotate(X, X, c.p.nb, c.p.nb, c.at<double>(c.L.mat3), c.p.batch, again, c.s));
  svqb_factor(c, again, c.L.mat2);
  HKP_CHECK(launch_rotate(X, X, c.p.nb, c.p.nb, c.at<double>(c.L.mat2), c.p.batch, again, c.s));
  HKP_CHECK(launch_set_identity(c.at<double>(c.L.mat3), c.p.nb, c.p.batch, ms, again, c.s));
}

// Rayleigh-Ritz on the span of X S (S in mat3, the SVQB factor or I): W = H X,
// the projection S^H (X^H W) S, its eigenpairs (theta, Q), T = S Q; then one
// pass over X and W gives X <- X T, the residual norms ||(W T)_j - theta_j
// (X T)_j|| and the next filter's first step alpha (W T - c X T) (FP32 for
// members filtered in FP32, else FP64 into W), without storing W T
void rayleigh_ritz(const Ctx& c, const int* active) {
  BlockDesc X = c.blk(c.L.X, c.p.nb), W = c.blk(c.L.W, c.p.nb);
  const long long ms = (long long)c.p.nb * c.p.nb;
  double* S = c.at<double>(c.L.mat3);
  double* M = c.at<double>(c.L.mat1);
  double* Q = c.at<double>(c.L.mat2);
  double* tmp = c.at<double>(c.L.mat4);
  apply_block(c, c.L.X, c.L.W, active);
  HKP_CHECK(launch_gram(X, W, 1, c.p.batch, c.at<double>(c.L.gram), M, active, c.s));
  HKP_CHECK(launch_small_gemm(M, 0, S, tmp, c.p.nb, c.p.batch, ms, 0, active, c.s));
  HKP_CHECK(launch_small_gemm(S, 1, tmp, M, c.p.nb, c.p.batch, ms, 1, active, c.s));
  HKP_CHECK(launch_heev(M, c.p.nb, c.p.batch, ms, c.at<double>(c.L.theta), tmp, 0, nullptr,
                        active, c.s));
  HKP_CHECK(launch_small_gemm(S, 0, tmp, Q, c.p.nb, c.p.batch, ms, 0, active, c.s));
  HKP_CHECK(launch_ritz(X, W, c.p.nb, c.at<double>(c.L.mat2), c.at<double>(c.L.theta),
                        c.at<double>(c.L.bounds),
                        c.p.product ? c.at<double>(c.L.roots) : nullptr, c.at<int>(c.L.act32),
                        c.p.mixed ? c.at<float>(c.L.A32) : nullptr, c.p.batch,
                        c.at<double>(c.L.rpart), c.at<double>(c.L.r2), active, c.s));
}

// k-step Lanczos per Hamiltonian: upper spectral bound (theta_max + beta_k)
void lanczos_bounds(const Ctx& c, std::vector<double>& bup) {
  const int B = c.p.batch;
  const long long n = c.p.n6, bs = c.bstride();
  double* vp = c.at<double>(c.L.X);
  double* v = c.at<double>(c.L.X) + 2 * n;
  double* w = c.at<double>(c.L.W);
  double* al = c.at<double>(c.L.lal);
  double* nrm = c.at<double>(c.L.lnrm);
  double* part = c.at<double>(c.L.lpart);
  HKP_CHECK(launch_random_block(v, n, 1, B, bs, 0x5eedULL, c.s));
  HKP_CHECK(launch_dots(v, v, n, B, bs, part, nrm, c.s));
  HKP_CHECK(launch_scale(v, n, B, bs, nrm, c.s));
  const int ksteps = (int)std::min<long long>(kLanczosSteps, std::max<long long>(2, n / 2));
  for (int j = 0; j < ksteps; ++j) {
    StencilLaunch a = base_launch(c, true, 1);
    a.in = v;
    a.in_bstride = bs;
    a.out = w;
    a.out_fp64 = 1;
    a.out_bstride = bs;
    c.ss->launch(a, c.consts, c.s, c.p.N, B);
    double* alj = al + 2LL * j * B;
    HKP_CHECK(launch_dots(v, w, n, B, bs, part, alj, c.s));
    HKP_CHECK(launch_lanczos_update(w, v, j > 0 ? vp : nullptr, n, B, bs, alj,
                                    j > 0 ? nrm + 2LL * j * B : nullptr, c.s));
    double* nj = nrm + 2LL * (j + 1) * B;
    HKP_CHECK(launch_dots(w, w, n, B, bs, part, nj, c.s));
    HKP_CHECK(launch_scale(w, n, B, bs, nj, c.s));
    double* t = vp;
    vp = v;
    v = w;
    w = t;
  }
  std::vector<double> hal(2 * (size_t)kLanczosSteps * B), hn(2 * (size_t)(kLanczosSteps + 1) * B);
  HKP_CHECK(hipMemcpyAsync(hal.data(), al, hal.size() * 8, hipMemcpyDeviceToHost, c.s));
  HKP_CHECK(hipMemcpyAsync(hn.data(), nrm, hn.size() * 8, hipMemcpyDeviceToHost, c.s));
  HKP_CHECK(hipStreamSynchronize(c.s));
  bup.resize(B);
  for (int b = 0; b < B; ++b) {
    std::vector<double> a(ksteps), b2(ksteps + 1, 0.0);
    for (int j = 0; j < ksteps; ++j) a[j] = hal[2 * ((size_t)j * B + b)];
    for (int j = 1; j <= ksteps; ++j) b2[j] = hn[2 * ((size_t)j * B + b)];
    double lo, hi;
    tridiag_extremes(a, b2, &lo, &hi);
    const double betak = std::sqrt(b2[ksteps]);
    bup[b] = hi + betak;
    if (!std::isfinite(bup[b])) throw std::runtime_error("Lanczos bound is not finite");
  }
}

struct Timer {
  hipEvent_t e0, e1;
  bool on;
  double acc = 0;
  explicit Timer(bool enable) : on(enable) {
    if (on) {
      HKP_CHECK(hipEventCreate(&e0));
      HKP_CHECK(hipEventCreate(&e1));
    }
  }
  ~Timer() {
    if (on) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
    }
  }
  void start(hipStream_t s) {
    if (on) HKP_CHECK(hipEventRecord(e0, s));
  }
  void stop(hipStream_t s) {
    if (on) HKP_CHECK(hipEventRecord(e1, s));
  }
  void collect() {
    if (!on) return;
    float ms = 0;
    HKP_CHECK(hipEventSynchronize(e1));
    HKP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    acc += ms * 1e-3;
  }
};

}  // namespace

Plan make_plan(const hkp_grid& g, const hkp_opts& o, int batch) {
  Plan p{};
  p.nx = g.nx;
  p.ny = g.ny;
  p.nz = g.nz;
  p.h = g.h_nm;
  p.N = (long long)g.nx * g.ny * g.nz;
  p.ncomp = (o.flags & HKP_FLAG_SPIN_FREE) ? 3 : 6;
  p.n6 = p.ncomp * p.N;
  p.batch = batch;
  p.nev = o.nev;
  p.nb = block_size(g, o);
  // degree 0: ramp 16 -> 32 -> m_max over the first outer iterations, so that
  // the amplification of the lowest components relative to the filter's cut
  // stays within the arithmetic's dynamic range while the interval settles.
  // m_max: 96 in FP64; in FP32 it grows with the block, 48 + nb within
  // [64, 96], since the per-iteration orthonormalisation and Rayleigh-Ritz cost
  // grows faster with the block than a filter step does (measured optimum 88 at
  // block 40 and 64 at block 16)
  p.degree_fixed = o.degree > 0;
  int m = o.degree > 0 ? o.degree
                       : (o.precision == HKP_PREC_MIXED ? std::min(96, std::max(64, 48 + p.nb)) : 96);
  if (m & 1) ++m;
  if (m > kKmax) m = kKmax;
  p.degree = m;
  p.mixed = o.precision == HKP_PREC_MIXED;
  p.product = (o.flags & HKP_FLAG_CHEB_PRODUCT) != 0;
  // the two-step pass carries the recurrence's old block
  p.two_step = p.mixed && !p.product && two_step_grid(p.nx, p.ncomp) && two_step_tuned(g, p.nb);
  return p;
}

int default_nb(int nev, long long n6) {
  int nb = nev + std::max(8, nev / 2);
  nb = (nb + 7) / 8 * 8;
  if (nb > HKP_NB_MAX) nb = HKP_NB_MAX;
  if (nb > n6) nb = (int)n6;
  return nb;
}

size_t plan_bytes(const Plan& p) { return make_layout(p).total; }

namespace {
thread_local hkp_iter_fn g_iter_fn = nullptr;
thread_local void* g_iter_user = nullptr;
}  // namespace

void set_iter_callback(hkp_iter_fn fn, void* user) {
  g_iter_fn = fn;
  g_iter_user = user;
}

int run_solve(const SolveArgs& A, hkp_stats* stats) {
  int n_sync = 0, n_graph = 0;   // host waits on the stream, graph replays
  const auto t_start = std::chrono::steady_clock::now();
  Ctx c;
  StencilStats sst;
  c.ss = &sst;
  c.active_members = A.plan.batch;
  c.p = A.plan;
  c.L = make_layout(c.p);
  c.ws = reinterpret_cast<char*>(A.workspace);
  c.s = reinterpret_cast<hipStream_t>(A.stream);
  c.field = A.B[0] != 0.0 || A.B[1] != 0.0 || A.B[2] != 0.0;
  c.field_z = A.B[2] != 0.0;
  c.strain = A.strain != nullptr;
  c.consts = make_consts(A.mat, c.p.h, A.B);
  c.p.st = A.st;
  const Plan& p = c.p;
  const bool eager = !(A.flags & HKP_FLAG_GRAPH);
  const char* tr = std::getenv("HKP_TRACE");
  const bool trace = tr && tr[0] == '1';   // HKP_TRACE=1: per iteration; 12: also per vector
  const bool timed = eager && stats != nullptr;
  Timer t_setup(timed), t_filter(timed), t_orth(timed), t_rr(timed), t_res(timed);
  sst.timed = timed;

  // ---- setup: on-site fields, phase tables, flags
  t_setup.start(c.s);
  HKP_CHECK(launch_fill_int(c.at<int>(c.L.status), p.batch + 1, 0, c.s));
  HKP_CHECK(launch_check_finite(A.V, (long long)p.batch * p.N, c.at<int>(c.L.status) + p.batch,
                                c.s));
  if (A.strain)
    HKP_CHECK(launch_check_finite(A.strain, 6LL * p.N, c.at<int>(c.L.status) + p.batch, c.s));
  int bad = 0;
  HKP_CHECK(hipMemcpyAsync(&bad, c.at<int>(c.L.status) + p.batch, 4, hipMemcpyDeviceToHost, c.s));
  HKP_CHECK(hipStreamSynchronize(c.s));
  ++n_sync;
  if (bad) {
    set_error("V or strain contains NaN or Inf");
    return HKP_E_ARG;
  }
  HKP_CHECK(launch_onsite(A.mat, p.nx, p.ny, p.nz, p.batch, A.V, p.N, A.strain,
                          c.at<double>(c.L.D64), p.mixed ? c.at<float>(c.L.D32) : nullptr,
                          6LL * p.N, c.s));
  if (c.field)
    HKP_CHECK(launch_phase_tables(p.nx, p.nz, p.h, A.B, c.at<double>(c.L.w64),
                                  c.at<double>(c.L.v64), c.at<float>(c.L.w32),
                                  c.at<float>(c.L.v32), c.s));
  HKP_CHECK(launch_fill_int(c.at<int>(c.L.flags), 8 * p.batch, 0, c.s));
  HKP_CHECK(launch_fill_int(c.at<int>(c.L.zero), 64, 0, c.s));
  HKP_CHECK(launch_fill_int(c.at<int>(c.L.active), p.batch, 1, c.s));
  HKP_CHECK(launch_fill_int(c.at<int>(c.L.act32), p.batch, p.mixed ? 1 : 0, c.s));
  HKP_CHECK(launch_fill_int(c.at<int>(c.L.act64), p.batch, p.mixed ? 0 : 1, c.s));
  HKP_CHECK(launch_fill_int(c.at<int>(c.L.lock), p.batch, 0, c.s));
  HKP_CHECK(launch_fill_int(c.at<int>(c.L.sw), p.batch, 0, c.s));
  HKP_CHECK(launch_worktable(c.control(), p.batch, p.nb, c.s));

  // ---- spectral bound
  std::vector<double> bup;
  if (A.bound_hint > 0.0 && p.batch == 1)
    bup.assign(1, A.bound_hint);
  else {
    lanczos_bounds(c, bup);
    ++n_sync;   // one wait for the Lanczos coefficients
  }
  {
    std::vector<double> hb(4 * (size_t)p.batch, 0.0);
    for (int b = 0; b < p.batch; ++b) hb[4 * b] = bup[b];
    HKP_CHECK(hipMemcpyAsync(c.at<double>(c.L.bounds), hb.data(), hb.size() * 8,
                             hipMemcpyHostToDevice, c.s));
    HKP_CHECK(hipStreamSynchronize(c.s));
    ++n_sync;
  }

  // ---- initial block: caller's X0 or random; SVQB; Rayleigh-Ritz
  const bool spin_free = (A.flags & HKP_FLAG_SPIN_FREE) != 0;
  if (spin_free) {
    // three-component orbital blocks
    double* X = c.at<double>(c.L.X);
    if (A.X0 && !(A.flags & HKP_FLAG_X0_NEV)) {
      HKP_CHECK(launch_orbital_to_internal(p.nx, p.ny, p.nz, p.nb * p.batch, A.X0, X, c.s));
    } else {
      HKP_CHECK(launch_random_block(X, p.n6, p.nb, p.batch, c.bstride(), A.seed, c.s));
      if (A.X0)
        for (int b = 0; b < p.batch; ++b)
          HKP_CHECK(launch_orbital_to_internal(
              p.nx, p.ny, p.nz, p.nev,
              static_cast<const double*>(A.X0) + 2 * (size_t)b * p.nev * 3 * p.N,
              X + 2 * (size_t)b * c.bstride(), c.s));
    }
  } else if (A.X0 && !(A.flags & HKP_FLAG_X0_NEV)) {
    // [batch][nb] vectors, contiguous in both layouts (member stride nb n6)
    HKP_CHECK(launch_abi_to_internal(p.nx, p.ny, p.nz, p.h, A.B, p.nb * p.batch, A.X0,
                                     c.at<double>(c.L.X), 0, c.s));
  } else if (A.X0) {
    // [batch][nev] given vectors lead each member's block; the rest are random
    HKP_CHECK(launch_random_block(c.at<double>(c.L.X), p.n6, p.nb, p.batch, c.bstride(),
                                  A.seed, c.s));
    for (int b = 0; b < p.batch; ++b)
      HKP_CHECK(launch_abi_to_internal(
          p.nx, p.ny, p.nz, p.h, A.B, p.nev,
          static_cast<const double*>(A.X0) + 2 * (size_t)b * p.nev * p.n6,
          c.at<double>(c.L.X) + 2 * (size_t)b * c.bstride(), 0, c.s));
  } else {
    HKP_CHECK(launch_random_block(c.at<double>(c.L.X), p.n6, p.nb, p.batch, c.bstride(),
                                  A.seed, c.s));
  }
  const int* act = c.at<int>(c.L.active);
  // the product form's roots for the next filter's degree (set when it changes)
  int roots_m = 0;
  auto prepare = [&](int m_next) {
    if (!p.product || m_next == roots_m) return;
    HKP_CHECK(launch_set_roots(c.at<double>(c.L.roots), leja_cheb_roots(m_next), m_next, c.s));
    roots_m = m_next;
  };
  const int m_first = p.degree_fixed ? p.degree : std::min(16, p.degree);
  prepare(m_first);
  orthonormalise(c, act);
  rayleigh_ritz(c, act);
  HKP_CHECK(launch_control(c.control(), p.batch, p.nb, p.nev, m_first, kKmax, A.tol, p.mixed,
                           !(A.flags & HKP_FLAG_NO_FP64_POLISH), !(A.flags & HKP_FLAG_NO_LOCK), 0,
                           c.s));
  t_setup.stop(c.s);
  t_setup.collect();

  long long n_hx64 = (long long)kLanczosSteps + p.nb, n_hx32 = 0;
  int iters = 0;
  std::vector<int> hflags(8 * (size_t)p.batch);
  auto read_flags = [&]() {
    HKP_CHECK(hipMemcpyAsync(hflags.data(), c.at<int>(c.L.flags), hflags.size() * 4,
                             hipMemcpyDeviceToHost, c.s));
    HKP_CHECK(hipStreamSynchronize(c.s));
    ++n_sync;
  };
  read_flags();
  {
    // the starting block must span nb directions: a breakdown of its first
    // orthonormalisation (a Gram eigenvalue below 1e-15 of the largest, e.g. an
    // X0 with repeated or dependent columns) is an error.  Later passes keep
    // their floor: a strongly filtered block may be nearly dependent.
    std::vector<int> st0(p.batch);
    HKP_CHECK(hipMemcpy(st0.data(), c.at<int>(c.L.status), p.batch * 4, hipMemcpyDeviceToHost));
    for (int b = 0; b < p.batch; ++b)
      if (st0[b]) {
        set_error("the initial block is rank deficient (member " + std::to_string(b) +
                  "): X0 columns must be linearly independent");
        return HKP_E_NUMERICAL;
      }
  }
  auto all_done = [&]() {
    for (int b = 0; b < p.batch; ++b)
      if (!hflags[8 * b]) return false;
    return true;
  };
  // the caller's progress callback (after read_flags); true: it asks to stop
  bool user_stop = false;
  auto report = [&](int done_iters) {
    if (!g_iter_fn || user_stop) return;
    const size_t nbb = (size_t)p.batch * p.nb;
    std::vector<double> th(nbb), res(nbb);
    HKP_CHECK(hipMemcpyAsync(th.data(), c.at<double>(c.L.theta), nbb * 8, hipMemcpyDeviceToHost,
                             c.s));
    HKP_CHECK(hipMemcpyAsync(res.data(), c.at<double>(c.L.r2), nbb * 8, hipMemcpyDeviceToHost,
                             c.s));
    HKP_CHECK(hipStreamSynchronize(c.s));
    ++n_sync;
    for (double& r : res) r = std::sqrt(r > 0.0 ? r : 0.0);
    std::vector<int32_t> nconv(p.batch), fp64(p.batch);
    for (int b = 0; b < p.batch; ++b) {
      nconv[b] = hflags[8 * b + 4];
      fp64[b] = hflags[8 * b + 1];
    }
    hkp_iter_info info{done_iters, p.batch, p.nb, p.nev, nconv.data(), fp64.data(), th.data(),
                       res.data()};
    user_stop = g_iter_fn(&info, g_iter_user) != 0;
  };
  auto degree_at = [&](int it) {   // it = 1, 2, ...
    if (p.degree_fixed) return p.degree;
    const int ramp = it == 1 ? 16 : (it == 2 ? 32 : p.degree);
    return std::min(ramp, p.degree);
  };
  int m_cur = degree_at(1);
  auto count_work = [&]() {
    c.active_members = 0;
    c.filtered_vectors = 0;
    for (int b = 0; b < p.batch; ++b) {
      if (hflags[8 * b]) continue;
      ++c.active_members;
      const int nf = p.nb - hflags[8 * b + 6];   // locked vectors are not filtered
      c.filtered_vectors += nf;
      const bool f32 = p.mixed && !hflags[8 * b + 1];
      (f32 ? n_hx32 : n_hx64) += (long long)nf * m_cur;
      n_hx64 += p.nb;
    }
  };

  auto iteration = [&](int it, bool single_path_known, bool f32_only, int m_next) {
    t_filter.start(c.s);
    if (!single_path_known) {
      if (p.mixed) filter32(c, c.at<int>(c.L.act32), m_cur);
      filter64(c, c.at<int>(c.L.act64), m_cur);
    } else if (f32_only) {
      filter32(c, act, m_cur);
    } else {
      filter64(c, act, m_cur);
    }
    t_filter.stop(c.s);
    t_orth.start(c.s);
    orthonormalise(c, act);
    t_orth.stop(c.s);
    t_rr.start(c.s);
    prepare(m_next);
    rayleigh_ritz(c, act);
    t_rr.stop(c.s);
    t_res.start(c.s);
    // stagnation toward the FP32 floor is judged after the degree ramp only
    // (during the ramp a slow decrease is the low degree's); graph replays
    // (it < 0) come after it
    const bool past_ramp = it < 0 || it > 2 || m_cur >= p.degree;
    HKP_CHECK(launch_control(c.control(), p.batch, p.nb, p.nev, m_next, kKmax, A.tol,
                             p.mixed,
                             !(A.flags & HKP_FLAG_NO_FP64_POLISH) && past_ramp,
                             !(A.flags & HKP_FLAG_NO_LOCK), it, c.s));
    t_res.stop(c.s);
  };

  // eager iterations: all of them, or in graph mode the ramp-up ones
  const int eager_iters = eager ? A.max_iter : (p.degree_fixed ? 0 : 2);
  {
    while (iters < std::min(A.max_iter, eager_iters) && !all_done() && !user_stop) {
      ++iters;
      m_cur = degree_at(iters);
      count_work();
      if (p.batch == 1) {
        const bool f32 = p.mixed && !hflags[1];
        iteration(iters, true, f32, degree_at(iters + 1));
      } else {
        iteration(iters, false, false, degree_at(iters + 1));
      }
      read_flags();
      report(iters);
      if (trace) {
        double bd[4];
        HKP_CHECK(hipMemcpy(bd, c.at<double>(c.L.bounds), 32, hipMemcpyDeviceToHost));
        std::fprintf(stderr, "[hkp] it %d m %d nconv %d lock %d rmax %.3e b %.6f a_cut %.6f a0 %.6f fp64 %d\n",
                     iters, m_cur, hflags[4], hflags[6], bd[3], bd[0], bd[1], bd[2], hflags[1]);
        if (tr[0] == '1' && tr[1] == '2') {   // HKP_TRACE=12: Ritz values and residuals
          std::vector<double> th(p.nb), r2(p.nb);
          HKP_CHECK(hipMemcpy(th.data(), c.at<double>(c.L.theta), p.nb * 8, hipMemcpyDeviceToHost));
          HKP_CHECK(hipMemcpy(r2.data(), c.at<double>(c.L.r2), p.nb * 8, hipMemcpyDeviceToHost));
          for (int j = 0; j < p.nb; ++j)
            std::fprintf(stderr, "[hkp]   %d %.12e %.3e\n", j, th[j], std::sqrt(r2[j]));
        }
      }
      t_filter.collect();
      t_orth.collect();
      t_rr.collect();
      t_res.collect();
      sst.collect();
    }
  }
  if (!eager && iters < A.max_iter && !all_done() && !user_stop) {
    // record a chunk of iterations once, replay until converged
    m_cur = p.degree;
    const int chunk = std::max(1, std::min(A.graph_chunk > 0 ? A.graph_chunk : 4, A.max_iter));
    // destroyed on every exit, an error thrown by a replay included
    struct Recorded {
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      ~Recorded() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
      }
    } rec;
    // byte accounting of a replay: the recorded chunk with every member active
    // and no vector locked (an upper estimate; the kernels skip on the device)
    const double bytes_before = sst.hx_bytes;
    c.active_members = p.batch;
    c.filtered_vectors = -1;
    HKP_CHECK(hipStreamBeginCapture(c.s, hipStreamCaptureModeThreadLocal));
    try {
      for (int k = 0; k < chunk; ++k) iteration(-1, false, false, p.degree);
    } catch (...) {
      hipGraph_t g2 = nullptr;
      (void)hipStreamEndCapture(c.s, &g2);
      if (g2) (void)hipGraphDestroy(g2);
      throw;
    }
    HKP_CHECK(hipStreamEndCapture(c.s, &rec.graph));
    const double chunk_bytes = sst.hx_bytes - bytes_before;
    sst.hx_bytes = bytes_before;
    HKP_CHECK(hipGraphInstantiate(&rec.exec, rec.graph, nullptr, nullptr, 0));
    while (iters < A.max_iter && !all_done() && !user_stop) {
      for (int k = 0; k < chunk; ++k) count_work();   // upper estimate per replay
      sst.hx_bytes += chunk_bytes;
      HKP_CHECK(hipGraphLaunch(rec.exec, c.s));
      ++n_graph;
      iters += chunk;
      read_flags();
      report(iters);
    }
  }

  // ---- outputs
  HKP_CHECK(launch_finish(c.at<double>(c.L.theta), c.at<double>(c.L.r2), p.nb, p.nev, p.batch,
                          A.eig, A.resid, c.s));
  const int npsi = (A.flags & HKP_FLAG_PSI_BLOCK) ? p.nb : p.nev;
  if (A.psi && spin_free)
    HKP_CHECK(launch_internal_to_orbital(p.nx, p.ny, p.nz, npsi, p.batch, c.at<double>(c.L.X),
                                         c.bstride(), A.psi, (long long)npsi * 3 * p.N, c.s));
  else if (A.psi)
    HKP_CHECK(launch_internal_to_abi(p.nx, p.ny, p.nz, p.h, A.B, npsi, p.batch,
                                     c.at<double>(c.L.X), c.bstride(), A.psi,
                                     (long long)npsi * p.n6, c.s));
  HKP_CHECK(hipStreamSynchronize(c.s));
  ++n_sync;
  int all = 1, minconv = p.nev, maxit = 0, sw = -1;
  for (int b = 0; b < p.batch; ++b) {
    all &= hflags[8 * b] != 0;
    minconv = std::min(minconv, hflags[8 * b + 4]);
    maxit = std::max(maxit, hflags[8 * b + 3]);
    if (hflags[8 * b + 1]) sw = sw < 0 ? hflags[8 * b + 5] : std::min(sw, hflags[8 * b + 5]);
  }
  if (stats) {
    stats->iters = std::max(0, maxit - 1);   // device count includes the initial Rayleigh-Ritz
    stats->n_converged = minconv;
    stats->n_hx_fp64 = n_hx64;
    stats->n_hx_fp32 = n_hx32;
    stats->fp64_switch_iter = p.mixed ? sw : -1;
    stats->nb = p.nb;
    stats->degree = p.degree;
    stats->t_setup = t_setup.acc;
    stats->t_filter = t_filter.acc;
    stats->t_orth = t_orth.acc;
    stats->t_rr = t_rr.acc;
    stats->t_resid = t_res.acc;
    stats->lambda_max_bound = bup.empty() ? 0.0 : bup[0];
    sst.collect();
    stats->hx_bytes = sst.hx_bytes;
    stats->n_stencil32 = sst.n32;
    stats->n_stencil64 = sst.n64;
    stats->t_stencil32 = sst.t32;
    stats->t_stencil64 = sst.t64;
    stats->bytes_stencil32 = sst.b32;
    stats->bytes_stencil64 = sst.b64;
    stats->n_stencil32x2 = sst.n32x2;
    stats->t_stencil32x2 = sst.t32x2;
    stats->bytes_stencil32x2 = sst.b32x2;
    stats->n_graph_launches = n_graph;
    stats->n_host_syncs = n_sync;
    stats->seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  }
  return all ? HKP_OK : HKP_W_NOT_CONVERGED;
}

// ---------------------------------------------------------------------------
// operator-level entry (tests): Y = alpha (H - shift) X + beta Y_old in the ABI layout
// ---------------------------------------------------------------------------
size_t apply_bytes(const hkp_grid& g, int nvec) {
  const size_t N = (size_t)g.nx * g.ny * g.nz;
  const size_t n6 = 6 * N;
  size_t b = 0;
  b += align_up(6 * N * 8) + align_up(6 * N * 4);                     // D64, D32
  b += align_up((size_t)g.nz * 16) + align_up((size_t)g.nz * g.nx * 16);
  b += align_up((size_t)g.nz * 8) + align_up((size_t)g.nz * g.nx * 8);
  b += 3 * align_up((size_t)nvec * n6 * 16);                          // X, Old, Y (FP64)
  b += align_up((size_t)nvec * n6 * 8);                               // X (FP32)
  return b;
}

int run_filter_step(const FilterArgs& A) {
  const hkp_grid& g = A.grid;
  const size_t N = (size_t)g.nx * g.ny * g.nz, n6 = 6 * N;
  char* ws = reinterpret_cast<char*>(A.workspace);
  hipStream_t s = reinterpret_cast<hipStream_t>(A.stream);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = ws + off;
    off += align_up(bytes);
    return p;
  };
  double* D64 = (double*)take(6 * N * 8);
  float* D32 = (float*)take(6 * N * 4);
  double* w64 = (double*)take((size_t)g.nz * 16);
  double* v64 = (double*)take((size_t)g.nz * g.nx * 16);
  float* w32 = (float*)take((size_t)g.nz * 8);
  float* v32 = (float*)take((size_t)g.nz * g.nx * 8);
  double* Xi = (double*)take((size_t)A.nvec * n6 * 16);
  double* Oi = (double*)take((size_t)A.nvec * n6 * 16);
  double* Yi = (double*)take((size_t)A.nvec * n6 * 16);
  float* Xf = (float*)take((size_t)A.nvec * n6 * 8);
  const bool fp64 = A.precision == HKP_PREC_FP64;
  const bool field = A.B[0] != 0.0 || A.B[1] != 0.0 || A.B[2] != 0.0;
  HKP_CHECK(launch_onsite(A.mat, g.nx, g.ny, g.nz, 1, A.V, 0, A.strain, D64, D32, 0, s));
  if (field) HKP_CHECK(launch_phase_tables(g.nx, g.nz, g.h_nm, A.B, w64, v64, w32, v32, s));
  HKP_CHECK(launch_abi_to_internal(g.nx, g.ny, g.nz, g.h_nm, A.B, A.nvec, A.X,
                                   fp64 ? (void*)Xi : (void*)Xf, fp64 ? 0 : 1, s));
  const bool has_old = A.Y_old != nullptr && A.beta != 0.0;
  if (has_old)
    HKP_CHECK(launch_abi_to_internal(g.nx, g.ny, g.nz, g.h_nm, A.B, A.nvec, A.Y_old, Oi, 0, s));
  StencilLaunch a{};
  a.nx = g.nx;
  a.ny = g.ny;
  a.nz = g.nz;
  a.nvec = A.nvec;
  a.batch = 1;
  a.in = fp64 ? (const void*)Xi : (const void*)Xf;
  a.old = has_old ? Oi : nullptr;
  a.old_fp64 = 1;
  a.out = Yi;
  a.out_fp64 = 1;
  a.D = fp64 ? (const void*)D64 : (const void*)D32;
  a.strain = A.strain != nullptr;
  if (field) {
    a.wtab = fp64 ? (const void*)w64 : (const void*)w32;
    a.vtab = fp64 ? (const void*)v64 : (const void*)v32;
    a.phase_general = A.B[2] != 0.0;
  }
  a.coef.alpha = A.alpha;
  a.coef.shift = A.shift;
  a.coef.beta = has_old ? A.beta : 0.0;
  a.tile_y = A.st.tile_y;
  a.vgroup = A.st.vgroup;
  a.dma = A.st.dma;
  a.zsplit = A.st.zsplit;
  a.fp64 = fp64;
  HKP_CHECK(launch_stencil(a, make_consts(A.mat, g.h_nm, A.B), s));
  HKP_CHECK(launch_internal_to_abi(g.nx, g.ny, g.nz, g.h_nm, A.B, A.nvec, 1, Yi, 0, A.Y, 0, s));
  return HKP_OK;
}

// two recurrence steps (FP32) in the ABI layout: X, Y_old -> Y1, Y2
size_t apply2_bytes(const hkp_grid& g, int nvec) {
  const size_t N = (size_t)g.nx * g.ny * g.nz;
  const size_t n6 = 6 * N;
  size_t b = 0;
  b += align_up(6 * N * 8) + align_up(6 * N * 4);                     // D64, D32
  b += align_up((size_t)g.nz * 16) + align_up((size_t)g.nz * g.nx * 16);
  b += align_up((size_t)g.nz * 8) + align_up((size_t)g.nz * g.nx * 8);
  b += 4 * align_up((size_t)nvec * n6 * 8);                           // X, Old, Y1, Y2 (FP32)
  b += align_up((size_t)nvec * n6 * 16);                              // FP64 staging
  b += align_up(256);                                                 // zeros
  return b;
}

int run_filter_step2(const Filter2Args& A, int* passes) {
  const hkp_grid& g = A.grid;
  const size_t N = (size_t)g.nx * g.ny * g.nz, n6 = 6 * N;
  char* ws = reinterpret_cast<char*>(A.workspace);
  hipStream_t s = reinterpret_cast<hipStream_t>(A.stream);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = ws + off;
    off += align_up(bytes);
    return p;
  };
  double* D64 = (double*)take(6 * N * 8);
  float* D32 = (float*)take(6 * N * 4);
  double* w64 = (double*)take((size_t)g.nz * 16);
  double* v64 = (double*)take((size_t)g.nz * g.nx * 16);
  float* w32 = (float*)take((size_t)g.nz * 8);
  float* v32 = (float*)take((size_t)g.nz * g.nx * 8);
  float* Xf = (float*)take((size_t)A.nvec * n6 * 8);
  float* Of = (float*)take((size_t)A.nvec * n6 * 8);
  float* Y1f = (float*)take((size_t)A.nvec * n6 * 8);
  float* Y2f = (float*)take((size_t)A.nvec * n6 * 8);
  double* Yd = (double*)take((size_t)A.nvec * n6 * 16);
  int* zero = (int*)take(256);
  const bool field = A.B[0] != 0.0 || A.B[1] != 0.0 || A.B[2] != 0.0;
  HKP_CHECK(launch_fill_int(zero, 64, 0, s));
  const StencilConsts<double> consts = make_consts(A.mat, g.h_nm, A.B);
  HKP_CHECK(launch_onsite(A.mat, g.nx, g.ny, g.nz, 1, A.V, 0, A.strain, D64, D32, 0, s));
  if (field) HKP_CHECK(launch_phase_tables(g.nx, g.nz, g.h_nm, A.B, w64, v64, w32, v32, s));
  HKP_CHECK(launch_abi_to_internal(g.nx, g.ny, g.nz, g.h_nm, A.B, A.nvec, A.X, Xf, 1, s));
  const bool has_old = A.Y_old != nullptr && A.beta[0] != 0.0;
  if (has_old)
    HKP_CHECK(launch_abi_to_internal(g.nx, g.ny, g.nz, g.h_nm, A.B, A.nvec, A.Y_old, Of, 1, s));

  Stencil2Launch t2{};
  t2.nx = g.nx;
  t2.ny = g.ny;
  t2.nz = g.nz;
  t2.nvec = A.nvec;
  t2.batch = 1;
  t2.in = Xf;
  t2.old = has_old ? Of : Xf;   // not read when beta[0] == 0
  t2.out1 = Y1f;
  t2.out2 = Y2f;
  t2.bstride = 0;
  t2.D = D32;
  t2.D_bstride = 0;
  t2.zero = zero;
  t2.strain = A.strain != nullptr;
  if (field) {
    t2.wtab = w32;
    t2.vtab = v32;
    t2.phase_general = A.B[2] != 0.0;
  }
  for (int i = 0; i < 3; ++i) {
    t2.host1[i] = i == 0 ? A.alpha[0] : (i == 1 ? A.shift[0] : (has_old ? A.beta[0] : 0.0));
    t2.host2[i] = i == 0 ? A.alpha[1] : (i == 1 ? A.shift[1] : A.beta[1]);
  }
  t2.tile_x = A.st.t2x > 0 ? A.st.t2x : 16;
  t2.tile_y = A.st.t2x > 0 ? A.st.t2y : (g.ny >= 12 ? 12 : 8);
  t2.vgroup = A.st.vgroup;
  if (two_step_grid(g.nx, 6) && stencil2_supported(t2)) {
    HKP_CHECK(launch_stencil2(t2, consts, s));
    *passes = 1;
  } else {
    // two one-step passes, FP32 throughout
    StencilLaunch a{};
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.nvec = A.nvec;
    a.batch = 1;
    a.D = D32;
    a.strain = A.strain != nullptr;
    if (field) {
      a.wtab = w32;
      a.vtab = v32;
      a.phase_general = A.B[2] != 0.0;
    }
    a.tile_y = A.st.tile_y;
    a.vgroup = A.st.vgroup;
    a.dma = A.st.dma;
    a.zsplit = A.st.zsplit;
    a.fp64 = 0;
    a.in = Xf;
    a.old = has_old ? Of : nullptr;
    a.old_fp64 = 0;
    a.out = Y1f;
    a.out_fp64 = 0;
    a.coef.alpha = A.alpha[0];
    a.coef.shift = A.shift[0];
    a.coef.beta = has_old ? A.beta[0] : 0.0;
    HKP_CHECK(launch_stencil(a, consts, s));
    a.in = Y1f;
    a.old = Xf;
    a.out = Y2f;
    a.coef.alpha = A.alpha[1];
    a.coef.shift = A.shift[1];
    a.coef.beta = A.beta[1];
    HKP_CHECK(launch_stencil(a, consts, s));
    *passes = 2;
  }
  const long long cnt = 2LL * A.nvec * (long long)n6;   // real scalars
  HKP_CHECK(launch_cast(Y1f, 0, Yd, 1, cnt, s));
  HKP_CHECK(launch_internal_to_abi(g.nx, g.ny, g.nz, g.h_nm, A.B, A.nvec, 1, Yd, 0, A.Y1, 0, s));
  HKP_CHECK(launch_cast(Y2f, 0, Yd, 1, cnt, s));
  HKP_CHECK(launch_internal_to_abi(g.nx, g.ny, g.nz, g.h_nm, A.B, A.nvec, 1, Yd, 0, A.Y2, 0, s));
  return HKP_OK;
}

// ---------------------------------------------------------------------------
// g-matrices: psi, r_a psi (16 vectors) -> H_0 of them, Z_b psi -> one Gram product
// L^H [L, H_0 L, Z psi] (16 x 44; L, the first 16 vectors of the block, is read twice
// by the same workgroup, the second time from cache).
// ---------------------------------------------------------------------------
constexpr int kGmSlots = 44;

size_t gmatrix_bytes(const hkp_grid& g) {
  const size_t N = (size_t)g.nx * g.ny * g.nz, n6 = 6 * N;
  return align_up(6 * N * 8) + align_up((size_t)kGmSlots * n6 * 16) +
         align_up(gram_partial_bytes(kGmSlots, (long long)n6, 1)) +
         align_up((size_t)16 * kGmSlots * 16);
}

int run_gmatrix(const GMatrixArgs& A) {
  const hkp_grid& g = A.grid;
  const size_t N = (size_t)g.nx * g.ny * g.nz, n6 = 6 * N;
  char* ws = reinterpret_cast<char*>(A.workspace);
  hipStream_t s = reinterpret_cast<hipStream_t>(A.stream);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = ws + off;
    off += align_up(bytes);
    return p;
  };
  double* D64 = (double*)take(6 * N * 8);
  double* buf = (double*)take((size_t)kGmSlots * n6 * 16);
  double* partial = (double*)take(gram_partial_bytes(kGmSlots, (long long)n6, 1));
  double* G = (double*)take((size_t)16 * kGmSlots * 16);
  const double B0[3] = {0.0, 0.0, 0.0};
  HKP_CHECK(launch_onsite(A.mat, g.nx, g.ny, g.nz, 1, A.V, 0, A.strain, D64, nullptr, 0, s));
  HKP_CHECK(launch_abi_to_internal(g.nx, g.ny, g.nz, g.h_nm, B0, 4, A.psi, buf, 0, s));
  HKP_CHECK(launch_position_weight(g.nx, g.ny, g.nz, g.h_nm, buf, s));
  StencilLaunch a{};
  a.nx = g.nx;
  a.ny = g.ny;
  a.nz = g.nz;
  a.nvec = 16;
  a.batch = 1;
  a.in = buf;
  a.old = nullptr;
  a.old_fp64 = 1;
  a.out = buf + 2 * 16 * n6;   // slot 16 (two doubles per complex entry)
  a.out_fp64 = 1;
  a.D = D64;
  a.strain = A.strain != nullptr;
  a.coef.alpha = 1.0;
  a.coef.shift = 0.0;
  a.coef.beta = 0.0;
  a.tile_y = A.st.tile_y;
  a.vgroup = A.st.vgroup;
  a.dma = A.st.dma;
  a.zsplit = A.st.zsplit;
  a.fp64 = 1;
  HKP_CHECK(launch_stencil(a, make_consts(A.mat, g.h_nm, B0), s));
  HKP_CHECK(launch_zeeman_derivative((long long)N, A.mat.kappa, buf, s));
  const BlockDesc L{buf, (long long)n6, 16, 0};
  const BlockDesc R{buf, (long long)n6, kGmSlots, 0};
  HKP_CHECK(launch_gram(L, R, 0, 1, partial, G, nullptr, s));
  HKP_CHECK(launch_gmatrix_post(G, A.out, s));
  return HKP_OK;
}

// translate a HIP failure into the ABI error code
int guarded(const std::function<int()>& f) {
  try {
    return f();
  } catch (const HipError& e) {
    set_error(e.what());
    return HKP_E_HIP;
  } catch (const std::exception& e) {
    set_error(e.what());
    return HKP_E_NUMERICAL;
  }
}

}  // namespace hkp
