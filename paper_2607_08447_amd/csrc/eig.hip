// Small dense Hermitian eigenproblems of the subspace iteration, one
// workgroup per matrix (nb <= 64), entirely on the device so that an outer
// iteration needs no host round trip and can be recorded in a hipGraph.
//
// Method: cyclic two-sided Jacobi with the round-robin (tournament) ordering,
// nb/2 disjoint rotations per round applied in parallel; complex rotations
// J = diag(1, e^{-i phi}) R(theta) reduce each 2x2 Hermitian block to a real
// symmetric one.  Converges quadratically to full FP64 accuracy.
//
// Modes
//   RR   (Rayleigh-Ritz):  A -> eigenvalues ascending + eigenvectors Q[v][w]
//   SVQB (orthonormaliser): S (Gram) -> T = D U diag(lambda)^-1/2 with
//         D = diag(S)^-1/2 and D S D = U diag(lambda) U^H; X T is orthonormal.
//
// Also: the control kernel that turns Ritz values and residuals into the
// convergence flags and the next Chebyshev filter coefficients.
#include "hkp_internal.h"

namespace hkp {

namespace {

constexpr int kJacThreads = 1024;
constexpr int kNBP = HKP_NB_MAX;   // padded size (even)

struct Rot {
  double c, s, er, ei;   // cos, sin, e^{i phi}
  int p, q;
};

// pair k of `round` for n players (n even): returns (p, q) with p < q
__device__ __forceinline__ void pair_of(int k, int round, int n, int* p, int* q) {
  const int m = n - 1;
  int a, b;
  if (k == 0) {
    a = m;
    b = round % m;
  } else {
    a = (round + k) % m;
    b = (round - k + m) % m;
  }
  *p = a < b ? a : b;
  *q = a < b ? b : a;
}

__global__ void __launch_bounds__(kJacThreads)
heev_kernel(double* A, int nb, long long mat_stride, double* evals, double* out, int mode,
            int* status, const int* active, int* again) {
  __shared__ double2 a[kNBP][kNBP + 1];
  __shared__ double2 v[kNBP][kNBP + 1];
  __shared__ Rot rot[kNBP / 2];
  __shared__ double dscale[kNBP];
  __shared__ double lam[kNBP];
  __shared__ int rank[kNBP];
  __shared__ double red[kJacThreads / 64];
  __shared__ int upair[(kNBP / 2) * (kNBP / 2 + 1) / 2];   // (P << 8) | Q, P <= Q
  __shared__ int any_rot;

  const int b = blockIdx.x;
  if (active && !active[b]) {
    if (again && threadIdx.x == 0) again[b] = 0;
    return;
  }
  const int tid = threadIdx.x;
  const int n = nb + (nb & 1);      // even number of players; the pad is decoupled
  const double2* Ab = reinterpret_cast<const double2*>(A + 2 * (long long)b * mat_stride);

  for (int t = tid; t < n * n; t += kJacThreads) {
    const int i = t / n, j = t % n;
    double2 x = make_double2(0, 0);
    if (i < nb && j < nb) x = Ab[(long long)i * nb + j];
    a[i][j] = x;
    v[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  // pair blocks on and above the block diagonal, row by row
  const int h = n / 2;
  const int nup = h * (h + 1) / 2;
  for (int t = tid; t < nup; t += kJacThreads) {
    int P = 0, rem = t;
    while (rem >= h - P) {
      rem -= h - P;
      ++P;
    }
    upair[t] = (P << 8) | (P + rem);
  }
  __syncthreads();
  if (mode == 1) {
    // D = diag(S)^-1/2, A <- D S D
    for (int i = tid; i < n; i += kJacThreads) {
      const double d = i < nb ? a[i][i].x : 1.0;
      dscale[i] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    }
    __syncthreads();
    for (int t = tid; t < n * n; t += kJacThreads) {
      const int i = t / n, j = t % n;
      const double s = dscale[i] * dscale[j];
      a[i][j].x *= s;
      a[i][j].y *= s;
    }
    __syncthreads();
  }
  for (int t = tid; t < n; t += kJacThreads) a[t][t].y = 0.0;
  // Frobenius norm: absolute threshold of the Rayleigh-Ritz mode (its
  // diagonal may be ~0 or negative); SVQB uses the relative test alone
  {
    double f = 0.0;
    for (int t = tid; t < n * n; t += kJacThreads) {
      const double2 x = a[t / n][t % n];
      f += x.x * x.x + x.y * x.y;
    }
    for (int off = 32; off > 0; off >>= 1) f += __shfl_down(f, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = f;
  }
  __syncthreads();
  double frob = 0.0;
  for (int k = 0; k < kJacThreads / 64; ++k) frob += red[k];
  frob = sqrt(frob);
  const double abs_thr = mode == 0 ? 1e-3 * 2.220446049250313e-16 * frob : 1e-300;
  __syncthreads();

  const double eps = 2.220446049250313e-16;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) any_rot = 0;
    __syncthreads();
    for (int round = 0; round < n - 1; ++round) {
      // rotation parameters, one thread per pair
      if (tid < n / 2) {
        int p, q;
        pair_of(tid, round, n, &p, &q);
        const double app = a[p][p].x, aqq = a[q][q].x;
        const double2 apq = a[p][q];
        const double mag = sqrt(apq.x * apq.x + apq.y * apq.y);
        Rot r;
        r.p = p;
        r.q = q;
        if (mag > eps * 0.5 * sqrt(fabs(app * aqq)) && mag > abs_thr) {
          const double zeta = (aqq - app) / (2.0 * mag);
          const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          r.c = 1.0 / sqrt(1.0 + t * t);
          r.s = t * r.c;
          r.er = apq.x / mag;
          r.ei = apq.y / mag;
          any_rot = 1;
        } else {
          r.c = 1.0;
          r.s = 0.0;
          r.er = 1.0;
          r.ei = 0.0;
        }
        rot[tid] = r;
      }
      __syncthreads();
      // A <- N^H A N and V <- V N with N block diagonal over the pairs,
      // N_k = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] on (p_k, q_k): every 2x2
      // block of A (pair P rows, pair Q columns) with P <= Q and every
      // (row, pair) slice of V is owned by one thread, so one phase updates
      // everything in place; the block (Q, P) is written as the conjugate
      // transpose of (P, Q), which keeps A exactly Hermitian
      {
        for (int t = tid; t < nup + n * h; t += kJacThreads) {
          if (t < nup) {
            const int P = upair[t] >> 8, Q = upair[t] & 255;
            const Rot rp = rot[P], rq = rot[Q];
            if (rp.s == 0.0 && rq.s == 0.0) continue;
            double2 a00 = a[rp.p][rq.p], a01 = a[rp.p][rq.q];
            double2 a10 = a[rp.q][rq.p], a11 = a[rp.q][rq.q];
            if (rq.s != 0.0) {
              // T = A_PQ N_Q: col p <- c col_p - s e^{-i phi} col_q, col q <- s col_p + c e^{-i phi} col_q
              const double2 e01 = make_double2(rq.er * a01.x + rq.ei * a01.y, rq.er * a01.y - rq.ei * a01.x);
              const double2 e11 = make_double2(rq.er * a11.x + rq.ei * a11.y, rq.er * a11.y - rq.ei * a11.x);
              const double2 t00 = make_double2(rq.c * a00.x - rq.s * e01.x, rq.c * a00.y - rq.s * e01.y);
              const double2 t01 = make_double2(rq.s * a00.x + rq.c * e01.x, rq.s * a00.y + rq.c * e01.y);
              const double2 t10 = make_double2(rq.c * a10.x - rq.s * e11.x, rq.c * a10.y - rq.s * e11.y);
              const double2 t11 = make_double2(rq.s * a10.x + rq.c * e11.x, rq.s * a10.y + rq.c * e11.y);
              a00 = t00; a01 = t01; a10 = t10; a11 = t11;
            }
            if (rp.s != 0.0) {
              // N_P^H T: row p <- c row_p - s e^{i phi} row_q, row q <- s row_p + c e^{i phi} row_q
              const double2 e10 = make_double2(rp.er * a10.x - rp.ei * a10.y, rp.er * a10.y + rp.ei * a10.x);
              const double2 e11 = make_double2(rp.er * a11.x - rp.ei * a11.y, rp.er * a11.y + rp.ei * a11.x);
              const double2 u00 = make_double2(rp.c * a00.x - rp.s * e10.x, rp.c * a00.y - rp.s * e10.y);
              const double2 u01 = make_double2(rp.c * a01.x - rp.s * e11.x, rp.c * a01.y - rp.s * e11.y);
              const double2 u10 = make_double2(rp.s * a00.x + rp.c * e10.x, rp.s * a00.y + rp.c * e10.y);
              const double2 u11 = make_double2(rp.s * a01.x + rp.c * e11.x, rp.s * a01.y + rp.c * e11.y);
              a00 = u00; a01 = u01; a10 = u10; a11 = u11;
            }
            if (P == Q) {
              // the rotated pair itself: annihilated entry exactly zero, real diagonal
              a01 = make_double2(0, 0);
              a10 = make_double2(0, 0);
              a00.y = 0.0;
              a11.y = 0.0;
            }
            a[rp.p][rq.p] = a00;
            a[rp.p][rq.q] = a01;
            a[rp.q][rq.p] = a10;
            a[rp.q][rq.q] = a11;
            if (P != Q) {
              a[rq.p][rp.p] = make_double2(a00.x, -a00.y);
              a[rq.q][rp.p] = make_double2(a01.x, -a01.y);
              a[rq.p][rp.q] = make_double2(a10.x, -a10.y);
              a[rq.q][rp.q] = make_double2(a11.x, -a11.y);
            }
          } else {
            const int u = t - nup;
            const Rot rq = rot[u % h];
            if (rq.s == 0.0) continue;
            const int i = u / h;
            const double2 xp = v[i][rq.p], xq = v[i][rq.q];
            const double2 eq = make_double2(rq.er * xq.x + rq.ei * xq.y, rq.er * xq.y - rq.ei * xq.x);
            v[i][rq.p] = make_double2(rq.c * xp.x - rq.s * eq.x, rq.c * xp.y - rq.s * eq.y);
            v[i][rq.q] = make_double2(rq.s * xp.x + rq.c * eq.x, rq.s * xp.y + rq.c * eq.y);
          }
        }
      }
      __syncthreads();
    }
    const int go = any_rot;
    __syncthreads();
    if (!go) break;
  }

  // eigenvalues (real diagonal) and ascending order (stable in index)
  for (int i = tid; i < n; i += kJacThreads) lam[i] = a[i][i].x;
  __syncthreads();
  for (int i = tid; i < nb; i += kJacThreads) {
    int rk = 0;
    const double li = lam[i];
    for (int j = 0; j < nb; ++j) {
      const double lj = lam[j];
      rk += (lj < li) || (lj == li && j < i);
    }
    rank[i] = rk;
  }
  __syncthreads();
  double* ev = evals + (long long)b * nb;
  double2* Ob = reinterpret_cast<double2*>(out + 2 * (long long)b * mat_stride);
  if (mode == 0) {
    for (int i = tid; i < nb; i += kJacThreads) ev[rank[i]] = lam[i];
    for (int t = tid; t < nb * nb; t += kJacThreads) {
      const int r = t / nb, c = t % nb;   // component r of eigenvector c
      Ob[(long long)r * nb + rank[c]] = v[r][c];
    }
  } else {
    // T[:, k] = D U[:, k] / sqrt(lambda_k) with a floor on tiny lambda
    double lmax = 0.0;
    for (int i = 0; i < nb; ++i) lmax = fmax(lmax, lam[i]);
    const double floor_ = lmax * 1e-15;
    int bad = 0;
    for (int i = tid; i < nb; i += kJacThreads) {
      ev[rank[i]] = lam[i];
      if (!(lam[i] > floor_)) bad = 1;
    }
    if (bad && status) atomicOr(status + b, 1);
    // a second orthonormalisation pass is needed only for an ill-conditioned
    // Gram matrix (one SVQB pass leaves an orthogonality error ~ eps kappa(S))
    if (again && tid == 0) {
      double lmin = lmax;
      for (int i = 0; i < nb; ++i) lmin = fmin(lmin, lam[i]);
      again[b] = !(lmin > 1e-4 * lmax);
    }
    for (int t = tid; t < nb * nb; t += kJacThreads) {
      const int r = t / nb, c = t % nb;
      const double l = lam[c] > floor_ ? lam[c] : floor_;
      const double s = dscale[r] / sqrt(l);
      Ob[(long long)r * nb + rank[c]] = make_double2(v[r][c].x * s, v[r][c].y * s);
    }
  }
}

// ---------------------------------------------------------------------------
// control: residual norms -> convergence; Ritz values -> next filter interval
// ---------------------------------------------------------------------------
__global__ void control_kernel(Control c, int nb, int nev, int degree, int kmax, double tol,
                               int mixed, int allow_switch, int allow_lock, int iter) {
  const int b = blockIdx.x;
  if (threadIdx.x != 0) return;
  int* fl = c.flags + 8 * b;
  const int was32 = c.act32[b];
  if (fl[0]) {   // done before this iteration: keep its results
    c.active[b] = 0;
    c.act32[b] = 0;
    c.act64[b] = 0;
    c.lock[b] = 0;
    c.sw[b] = 0;
    return;
  }
  const double* th = c.theta + (long long)b * nb;
  const double* r2 = c.r2 + (long long)b * nb;
  double* bd = c.bounds + 4 * b;
  int nconv = 0;
  double rmax = 0.0;
  for (int j = 0; j < nev; ++j) {
    const double r = sqrt(r2[j]);
    if (r <= tol) ++nconv;
    rmax = fmax(rmax, r);
  }
  const int it = fl[3] + 1;   // outer iterations so far (counted on the device)
  fl[3] = it;
  fl[4] = nconv;
  if (nconv == nev) fl[0] = 1;
  // mixed precision: leave the FP32 filter once it can no longer reduce the
  // residual.  FP32 rounding of the filtered block leaves a residual floor of
  // a few FP32 ulps of the spectral radius (measured: ~3 eps32 |H|); stagnation
  // (less than a 30% decrease on two consecutive iterations) is only counted
  // within 30 eps32 |H| of the floor
  if (mixed && allow_switch && !fl[1] && !fl[0]) {
    const double prev = bd[3];
    const double near_floor = 30.0 * 5.96e-8 * bd[0];
    if (iter == 0 && rmax < near_floor && tol < 3.0 * 5.96e-8 * bd[0]) {
      // a restart that already starts near the floor, with a target below it,
      // gains nothing from FP32 filtering: FP64 from the first iteration
      fl[1] = 1;
      fl[5] = 1;
    } else {
      if (prev > 0.0 && rmax > 0.7 * prev && rmax < near_floor) fl[2] += 1; else fl[2] = 0;
      if (fl[2] >= 2) {
        fl[1] = 1;
        fl[5] = it + 1;
      }
    }
  }
  bd[3] = rmax;
  c.active[b] = fl[0] ? 0 : 1;
  c.act32[b] = (!fl[0] && mixed && !fl[1]) ? 1 : 0;
  c.act64[b] = (!fl[0] && !(mixed && !fl[1])) ? 1 : 0;
  c.sw[b] = (was32 && c.act64[b]) ? 1 : 0;
  // soft locking: the leading run of converged states, whole Kramers pairs,
  // is left out of the next filter (it stays in the block, so orthonormalisation
  // and Rayleigh-Ritz still see it, and it is released if its residual grows)
  int lead = 0;
  while (allow_lock && lead < nev && sqrt(r2[lead]) <= tol) ++lead;
  c.lock[b] = fl[0] ? 0 : (lead & ~1);
  fl[6] = c.lock[b];
  // next filter: damp [a_cut, b_up], scaled to 1 at a0 = lowest Ritz value
  const double bup = bd[0];
  const double a0 = th[0];
  double acut = th[nb - 1], e, cc, sigma1;
  cheb_interval(bup, a0, acut, &e, &cc, &sigma1);
  bd[1] = acut;
  bd[2] = a0;
  double* co = c.coef + (long long)b * kmax * 4;
  if (c.roots) {
    // product form: step k is (H - r_k) / (a0 - r_k), r_k the k-th root (Leja
    // order) mapped onto [a_cut, b_up]; degree = the next filter's m
    for (int k = 0; k < degree && k < kmax; ++k) {
      const double r = cc + e * c.roots[k];
      co[4 * k] = 1.0 / (a0 - r);
      co[4 * k + 1] = r;
      co[4 * k + 2] = 0.0;
    }
    return;
  }
  double sig = sigma1;
  co[0] = sigma1 / e;
  co[1] = cc;
  co[2] = 0.0;
  for (int k = 1; k < degree && k < kmax; ++k) {
    const double sn = 1.0 / (2.0 / sigma1 - sig);
    co[4 * k] = 2.0 * sn / e;
    co[4 * k + 1] = cc;
    co[4 * k + 2] = -sig * sn;
    sig = sn;
  }
}

// prefix sums of the vectors each member still has to process: the stencil
// launches map their live workgroups onto these so that converged members and
// locked vectors leave no XCD idle
__global__ void worktable_kernel(Control c, int batch, int nb) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int* t32 = c.work;
  int* t64 = c.work + (batch + 1);
  int* tall = c.work + 2 * (batch + 1);
  int s32 = 0, s64 = 0, sall = 0;
  for (int b = 0; b < batch; ++b) {
    t32[b] = s32;
    t64[b] = s64;
    tall[b] = sall;
    const int nf = nb - c.lock[b];
    s32 += c.act32[b] ? nf : 0;
    s64 += c.act64[b] ? nf : 0;
    sall += c.active[b] ? nb : 0;
  }
  t32[batch] = s32;
  t64[batch] = s64;
  tall[batch] = sall;
}

// eig[b][j] = theta[b][j], resid[b][j] = sqrt(r2[b][j]) for j < nev
__global__ void finish_kernel(const double* theta, const double* r2, int nb, int nev, int batch,
                              double* eig, double* resid) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= batch * nev) return;
  const int b = t / nev, j = t % nev;
  if (eig) eig[t] = theta[(long long)b * nb + j];
  if (resid) resid[t] = sqrt(r2[(long long)b * nb + j]);
}

__global__ void finite_kernel(const double* x, long long count, int* flag) {
  int bad = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    bad |= !isfinite(x[i]);
  if (bad) atomicOr(flag, 1);
}

__global__ void fill_int_kernel(int* p, int count, int value) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = value;
}

}  // namespace

hipError_t launch_finish(const double* theta, const double* r2, int nb, int nev, int batch,
                         double* eig, double* resid, hipStream_t s) {
  const int cnt = batch * nev;
  finish_kernel<<<(cnt + 255) / 256, 256, 0, s>>>(theta, r2, nb, nev, batch, eig, resid);
  return hipGetLastError();
}

hipError_t launch_check_finite(const double* x, long long count, int* flag, hipStream_t s) {
  long long g = (count + 255) / 256;
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  finite_kernel<<<(unsigned)g, 256, 0, s>>>(x, count, flag);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int count, int value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  fill_int_kernel<<<(count + 255) / 256, 256, 0, s>>>(p, count, value);
  return hipGetLastError();
}

namespace {

// small complex products of the block step, one workgroup per member, operands
// in LDS: C = op(A) B (op: A, or A^H), or with unit set C = I.  Row-major nb x nb.
constexpr int kGemmThreads = 256;

__global__ void __launch_bounds__(kGemmThreads)
small_gemm_kernel(const double* A, int adj, const double* B, double* C, int nb,
                  long long mat_stride, int herm, const int* active) {
  const int b = blockIdx.x;
  if (active && !active[b]) return;
  __shared__ double2 sa[kNBP * kNBP], sb[kNBP * kNBP];
  const double2* Ab = reinterpret_cast<const double2*>(A + 2 * (long long)b * mat_stride);
  const double2* Bb = reinterpret_cast<const double2*>(B + 2 * (long long)b * mat_stride);
  double2* Cb = reinterpret_cast<double2*>(C + 2 * (long long)b * mat_stride);
  const int nn = nb * nb;
  for (int t = threadIdx.x; t < nn; t += kGemmThreads) {
    sa[t] = Ab[t];
    sb[t] = Bb[t];
  }
  __syncthreads();
  // C[i][j] = sum_k op(A)[i][k] B[k][j]; op(A)[i][k] = A[i][k] or conj(A[k][i])
  auto entry = [&](int i, int j) {
    double re = 0.0, im = 0.0;
    for (int k = 0; k < nb; ++k) {
      const double2 a = adj ? make_double2(sa[k * nb + i].x, -sa[k * nb + i].y) : sa[i * nb + k];
      const double2 v = sb[k * nb + j];
      re = fma(a.x, v.x, fma(-a.y, v.y, re));
      im = fma(a.x, v.y, fma(a.y, v.x, im));
    }
    return make_double2(re, im);
  };
  for (int t = threadIdx.x; t < nn; t += kGemmThreads) {
    const int i = t / nb, j = t - (t / nb) * nb;
    double2 c = entry(i, j);
    if (herm) {   // the Hermitian part (the product is Hermitian up to rounding)
      const double2 d = entry(j, i);
      c = make_double2(0.5 * (c.x + d.x), 0.5 * (c.y - d.y));
      if (i == j) c.y = 0.0;
    }
    Cb[t] = c;
  }
}

__global__ void set_roots_kernel(double* dst, RootTable t, int m) {
  for (int k = threadIdx.x; k < m; k += blockDim.x) dst[k] = t.x[k];
}

__global__ void set_identity_kernel(double* C, int nb, long long mat_stride, const int* active) {
  const int b = blockIdx.x;
  if (active && !active[b]) return;
  double2* Cb = reinterpret_cast<double2*>(C + 2 * (long long)b * mat_stride);
  for (int t = threadIdx.x; t < nb * nb; t += blockDim.x)
    Cb[t] = make_double2(t / nb == t % nb ? 1.0 : 0.0, 0.0);
}

}  // namespace

hipError_t launch_small_gemm(const double* A, int adj, const double* B, double* C, int nb,
                             int batch, long long mat_stride, int herm, const int* active,
                             hipStream_t s) {
  if (nb > HKP_NB_MAX || nb < 1 || C == A || C == B) return hipErrorInvalidValue;
  small_gemm_kernel<<<batch, kGemmThreads, 0, s>>>(A, adj, B, C, nb, mat_stride, herm, active);
  return hipGetLastError();
}

hipError_t launch_set_roots(double* dst, const RootTable& t, int m, hipStream_t s) {
  if (m < 1 || m > kMaxDegree) return hipErrorInvalidValue;
  set_roots_kernel<<<1, 256, 0, s>>>(dst, t, m);
  return hipGetLastError();
}

hipError_t launch_set_identity(double* C, int nb, int batch, long long mat_stride,
                               const int* active, hipStream_t s) {
  set_identity_kernel<<<batch, 256, 0, s>>>(C, nb, mat_stride, active);
  return hipGetLastError();
}

hipError_t launch_heev(double* A, int nb, int batch, long long mat_stride, double* evals,
                       double* out, int mode, int* status, const int* active, hipStream_t s,
                       int* again) {
  if (nb > HKP_NB_MAX || nb < 1) return hipErrorInvalidValue;
  heev_kernel<<<batch, kJacThreads, 0, s>>>(A, nb, mat_stride, evals, out, mode, status, active,
                                            again);
  return hipGetLastError();
}

hipError_t launch_control(const Control& c, int batch, int nb, int nev, int degree, int kmax,
                          double tol, int mixed, int allow_switch, int allow_lock, int iter,
                          hipStream_t s) {
  control_kernel<<<batch, 64, 0, s>>>(c, nb, nev, degree, kmax, tol, mixed, allow_switch,
                                      allow_lock, iter);
  worktable_kernel<<<1, 64, 0, s>>>(c, batch, nb);
  return hipGetLastError();
}

hipError_t launch_worktable(const Control& c, int batch, int nb, hipStream_t s) {
  worktable_kernel<<<1, 64, 0, s>>>(c, batch, nb);
  return hipGetLastError();
}

}  // namespace hkp
