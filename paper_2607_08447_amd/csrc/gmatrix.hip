// g-matrices of the double dot's Kramers doublets and the effective two-spin
// model (paper Sec. III: Eqs. HB, J_QD, J_anis).
//
// The g-matrix of a doublet {u1, u2} comes from the field derivative of the
// Hamiltonian at B = 0 restricted to it, M_b = <u|dH/dB_b|u> = (mu_B / 2)
// sum_a g_ab sigma_a.  With straight-link Peierls phases in the symmetric gauge
// about r0 (the two-step links of the mixed derivatives average to the straight
// one at first order in B) the derivative is
//     dH/dB_b = Z_b + i (e / 2 hbar) eps_bcd (R - r0)_c H_0 (R - r0)_d,
// Z_b the on-site Zeeman matrix per tesla and R the position.  So everything
// needed for four states psi_i comes from one B = 0 stencil apply to the 16
// vectors {psi_i, R_x psi_i, R_y psi_i, R_z psi_i} and one Gram product of those
// 16 against themselves, their images under H_0 and Z_b psi_i (16 x 44).  The
// origin of each doublet's gauge is its own centre of charge, which enters the
// small matrices only.  Everything after the Gram product is 4 x 4 algebra done
// by a few threads of one workgroup.
#include <hip/hip_runtime.h>

#include "hkp_internal.h"

namespace hkp {

namespace {

constexpr int kT = 256;

__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) {
  return make_double2(a.x * s, a.y * s);
}
__device__ __forceinline__ double2 times_i(double2 a) { return make_double2(-a.y, a.x); }

__device__ __forceinline__ double levi(int a, int b, int c) {
  if (a == b || b == c || a == c) return 0.0;
  return ((b - a + 3) % 3 == 1) ? 1.0 : -1.0;
}

// Cyclic Jacobi for a small Hermitian matrix: A is destroyed, w ascending,
// column k of V the eigenvector of w[k].  A pivot rotation first turns A_pq
// real by a phase on column q, then applies the real rotation that zeroes it.
template <int N>
__device__ void jacobi_herm(double2 (&A)[N][N], double2 (&V)[N][N], double (&w)[N]) {
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) V[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int p = 0; p < N; ++p) {
      diag += A[p][p].x * A[p][p].x;
      for (int q = p + 1; q < N; ++q) off += A[p][q].x * A[p][q].x + A[p][q].y * A[p][q].y;
    }
    if (off == 0.0 || off <= 1e-34 * diag) break;
    for (int p = 0; p < N; ++p) {
      for (int q = p + 1; q < N; ++q) {
        const double ap = hypot(A[p][q].x, A[p][q].y);
        if (ap == 0.0) continue;
        const double2 ph = cscale(A[p][q], 1.0 / ap);
        const double2 em = cconj(ph);
        const double th = (A[q][q].x - A[p][p].x) / (2.0 * ap);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < N; ++k) {
          const double2 akp = A[k][p], akq = A[k][q];
          A[k][p] = csub(cscale(akp, c), cscale(cmul(em, akq), s));
          A[k][q] = cadd(cscale(akp, s), cscale(cmul(em, akq), c));
          const double2 vkp = V[k][p], vkq = V[k][q];
          V[k][p] = csub(cscale(vkp, c), cscale(cmul(em, vkq), s));
          V[k][q] = cadd(cscale(vkp, s), cscale(cmul(em, vkq), c));
        }
        for (int k = 0; k < N; ++k) {
          const double2 apk = A[p][k], aqk = A[q][k];
          A[p][k] = csub(cscale(apk, c), cscale(cmul(ph, aqk), s));
          A[q][k] = cadd(cscale(apk, s), cscale(cmul(ph, aqk), c));
        }
        A[p][q] = A[q][p] = make_double2(0.0, 0.0);
        A[p][p].y = 0.0;
        A[q][q].y = 0.0;
      }
    }
  }
  for (int i = 0; i < N; ++i) w[i] = A[i][i].x;
  for (int i = 0; i < N; ++i) {   // selection sort, columns of V along
    int m = i;
    for (int j = i + 1; j < N; ++j)
      if (w[j] < w[m]) m = j;
    if (m != i) {
      const double tw = w[i];
      w[i] = w[m];
      w[m] = tw;
      for (int k = 0; k < N; ++k) {
        const double2 tv = V[k][i];
        V[k][i] = V[k][m];
        V[k][m] = tv;
      }
    }
  }
}

// rotation by angle about the unit vector n (right-hand rule)
__device__ void rotation(const double n[3], double angle, double R[3][3]) {
  const double s = sin(angle), c = cos(angle), v = 1.0 - c;
  R[0][0] = c + v * n[0] * n[0];
  R[0][1] = v * n[0] * n[1] - s * n[2];
  R[0][2] = v * n[0] * n[2] + s * n[1];
  R[1][0] = v * n[1] * n[0] + s * n[2];
  R[1][1] = c + v * n[1] * n[1];
  R[1][2] = v * n[1] * n[2] - s * n[0];
  R[2][0] = v * n[2] * n[0] - s * n[1];
  R[2][1] = v * n[2] * n[1] + s * n[0];
  R[2][2] = c + v * n[2] * n[2];
}

__device__ void matvec3(const double A[3][3], const double x[3], double y[3]) {
  for (int i = 0; i < 3; ++i) y[i] = A[i][0] * x[0] + A[i][1] * x[1] + A[i][2] * x[2];
}

// a proper rotation R with R n = z: about n x z by the angle between n and z
// (the lab frame for n = 0)
__device__ void qubit_frame(const double v[3], double R[3][3]) {
  const double nn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R[i][j] = i == j ? 1.0 : 0.0;
  if (!(nn > 0.0)) return;
  const double n[3] = {v[0] / nn, v[1] / nn, v[2] / nn};
  const double ax[3] = {n[1], -n[0], 0.0};   // n x z
  const double s = sqrt(ax[0] * ax[0] + ax[1] * ax[1]), c = n[2];
  if (s < 1e-300) {
    if (c < 0.0) {
      R[1][1] = -1.0;
      R[2][2] = -1.0;
    }
    return;
  }
  const double u[3] = {ax[0] / s, ax[1] / s, 0.0};
  rotation(u, atan2(s, c), R);
}

// [v][c][p] internal block (LS, p = (z ny + y) nx + x): slots 4 (a + 1) + v <- r_a psi_v,
// r about the box centre
__global__ void __launch_bounds__(kT)
position_weight_kernel(int nx, int ny, int nz, double h, double2* buf) {
  const long long N = (long long)nx * ny * nz;
  const long long p = (long long)blockIdx.x * kT + threadIdx.x;
  const int v = blockIdx.y;
  if (p >= N) return;
  const int x = (int)(p % nx), y = (int)((p / nx) % ny), z = (int)(p / ((long long)nx * ny));
  const double r[3] = {(x - 0.5 * (nx - 1)) * h, (y - 0.5 * (ny - 1)) * h,
                       (z - 0.5 * (nz - 1)) * h};
  const long long n6 = 6 * N;
  for (int c = 0; c < 6; ++c) {
    const double2 val = buf[v * n6 + c * N + p];
    for (int a = 0; a < 3; ++a) buf[(4 * (a + 1) + v) * n6 + c * N + p] = cscale(val, r[a]);
  }
}

// slots 32 + 4 b + v <- Z_b psi_v, Z_b = mu_B [(3 kappa - 1) 1 (x) L_b + sigma_b (x) 1]
// in the |L S> basis (component 3 s + o), (L_b)_oo' = -i eps_boo'
__global__ void __launch_bounds__(kT)
zeeman_derivative_kernel(long long N, double g_orb, double2* buf) {
  const long long p = (long long)blockIdx.x * kT + threadIdx.x;
  const int v = blockIdx.y;
  if (p >= N) return;
  const long long n6 = 6 * N;
  double2 ps[2][3];
  for (int s = 0; s < 2; ++s)
    for (int o = 0; o < 3; ++o) ps[s][o] = buf[v * n6 + (3 * s + o) * N + p];
  for (int b = 0; b < 3; ++b) {
    double2* out = buf + (32 + 4 * b + v) * n6 + p;
    for (int s = 0; s < 2; ++s) {
      for (int o = 0; o < 3; ++o) {
        double2 orb = make_double2(0.0, 0.0);
        for (int o2 = 0; o2 < 3; ++o2) {
          const double e = levi(b, o, o2);
          if (e != 0.0) orb = cadd(orb, cscale(ps[s][o2], e));
        }
        orb = cscale(times_i(orb), -g_orb);   // -i eps psi, times mu_B (3 kappa - 1)
        double2 spin;
        if (b == 0) {
          spin = ps[1 - s][o];
        } else if (b == 1) {
          spin = s == 0 ? cscale(times_i(ps[1][o]), -1.0) : times_i(ps[0][o]);
        } else {
          spin = s == 0 ? ps[0][o] : cscale(ps[1][o], -1.0);
        }
        out[(3 * s + o) * N] = cadd(orb, cscale(spin, kMuB));
      }
    }
  }
}

// 4 x 4 blocks of the Gram product G = L^H [L, H_0 L, Z psi] (16 x 44, row-major):
// slot 4 c + i is r_c psi_i (c = 0: psi itself)
__device__ __forceinline__ double2 gW(const double2* G, int c, int i, int d, int j) {
  return G[(4 * c + i) * 44 + 16 + 4 * d + j];   // <r_c psi_i | H_0 | r_d psi_j>
}
__device__ __forceinline__ double2 gX(const double2* G, int a, int i, int j) {
  return G[i * 44 + 4 * (a + 1) + j];            // <psi_i | r_a | psi_j>
}
__device__ __forceinline__ double2 gZ(const double2* G, int b, int i, int j) {
  return G[i * 44 + 32 + 4 * b + j];             // <psi_i | Z_b | psi_j>
}

__device__ void sym_g(const double g[3][3], double out[3][3]) {
  double2 A[3][3], V[3][3];
  double w[3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += g[k][i] * g[k][j];
      A[i][j] = make_double2(s, 0.0);
    }
  jacobi_herm<3>(A, V, w);
  const double det = g[0][0] * (g[1][1] * g[2][2] - g[1][2] * g[2][1]) -
                     g[0][1] * (g[1][0] * g[2][2] - g[1][2] * g[2][0]) +
                     g[0][2] * (g[1][0] * g[2][1] - g[1][1] * g[2][0]);
  const double sg = det < 0.0 ? -1.0 : 1.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += V[i][k].x * sqrt(fmax(w[k], 0.0)) * V[j][k].x;
      out[i][j] = sg * s;
    }
}

// the doublet bases as columns over the four input states: bonding, antibonding,
// then the localised left and right doublets (columns of C)
__device__ void doublet_basis(int k, const double2 (&C)[4][4], double2 (&U)[4][2]) {
  const double2 zero = make_double2(0.0, 0.0), one = make_double2(1.0, 0.0);
  for (int i = 0; i < 4; ++i)
    for (int m = 0; m < 2; ++m) U[i][m] = k < 2 ? ((i == 2 * k + m) ? one : zero) : C[i][2 * (k - 2) + m];
}

// Phases, one workgroup: thread 0 localises the dots (4 x 4 Jacobi); four threads
// take the doublets' centres; twelve take one (doublet, field direction) column of
// g each; four take the symmetric tensors.
__global__ void gmatrix_post_kernel(const double2* __restrict__ Gg, hkp_gmatrix_result* out) {
  __shared__ double2 G[16 * 44];   // the whole Gram block, staged once by the workgroup
  __shared__ double2 sC[4][4];
  __shared__ double sR0[4][3], sg[4][3][3];
  const int t = threadIdx.x;
  for (int i = t; i < 16 * 44; i += blockDim.x) G[i] = Gg[i];
  __syncthreads();
  if (t == 0) {   // the dots' doublets: eigenvectors of x within the span, lower x first
    double2 Xx[4][4], C[4][4];
    double wx[4];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j)
        Xx[i][j] = cscale(cadd(gX(G, 0, i, j), cconj(gX(G, 0, j, i))), 0.5);
    jacobi_herm<4>(Xx, C, wx);
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) sC[i][j] = C[i][j];
    for (int i = 0; i < 4; ++i) out->E_eV[i] = gW(G, 0, i, 0, i).x;
  }
  __syncthreads();
  if (t < 4) {   // centre of charge of doublet t: tr(U^H X_a U) / 2
    double2 U[4][2];
    doublet_basis(t, sC, U);
    for (int a = 0; a < 3; ++a) {
      double s = 0.0;
      for (int m = 0; m < 2; ++m)
        for (int i = 0; i < 4; ++i)
          for (int j = 0; j < 4; ++j) s += cmul(cconj(U[i][m]), cmul(gX(G, a, i, j), U[j][m])).x;
      sR0[t][a] = 0.5 * s;
      out->centre_nm[t][a] = 0.5 * s;
    }
  }
  __syncthreads();
  if (t < 12) {   // column b of the g-matrix of doublet k
    const int k = t / 3, b = t % 3;
    double2 U[4][2];
    doublet_basis(k, sC, U);
    const double r0[3] = {sR0[k][0], sR0[k][1], sR0[k][2]};
    // D_b on the four states, gauge origin r0
    double2 D[4][4];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        double2 orb = make_double2(0.0, 0.0);
        for (int c = 0; c < 3; ++c)
          for (int d = 0; d < 3; ++d) {
            const double e = levi(b, c, d);
            if (e == 0.0) continue;
            double2 w = gW(G, c + 1, i, d + 1, j);
            w = csub(w, cscale(gW(G, 0, i, d + 1, j), r0[c]));
            w = csub(w, cscale(gW(G, c + 1, i, 0, j), r0[d]));
            orb = cadd(orb, cscale(w, e));
          }
        D[i][j] = cadd(gZ(G, b, i, j), cscale(times_i(orb), 0.5 * kEoverHbar));
      }
    // M_b = U^H D_b U
    double2 M[2][2];
    for (int m = 0; m < 2; ++m)
      for (int n = 0; n < 2; ++n) {
        double2 s2 = make_double2(0.0, 0.0);
        for (int i = 0; i < 4; ++i)
          for (int j = 0; j < 4; ++j) s2 = cadd(s2, cmul(cconj(U[i][m]), cmul(D[i][j], U[j][n])));
        M[m][n] = s2;
      }
    // g_ab = Re tr(sigma_a M_b) / mu_B: tr(sigma_x M) = M01 + M10,
    // tr(sigma_y M) = i (M01 - M10), tr(sigma_z M) = M00 - M11
    sg[k][0][b] = (M[0][1].x + M[1][0].x) / kMuB;
    sg[k][1][b] = (M[1][0].y - M[0][1].y) / kMuB;
    sg[k][2][b] = (M[0][0].x - M[1][1].x) / kMuB;
    out->kramers[k][b] = (M[0][0].x + M[1][1].x) / kMuB;
  }
  __syncthreads();
  if (t < 4) {
    double g[3][3], gs[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) g[a][b] = sg[t][a][b];
    sym_g(g, gs);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        out->g[t][a][b] = g[a][b];
        out->g_sym[t][a][b] = gs[a][b];
      }
  }
  if (t == 0) {
    double E[4];
    for (int i = 0; i < 4; ++i) E[i] = gW(G, 0, i, 0, i).x;
    const double delta = 0.5 * (E[2] + E[3]) - 0.5 * (E[0] + E[1]);
    out->delta_eV = delta;
    out->t_eV = fabs(delta) / sqrt(2.0);
    double dd = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double q = sR0[3][a] - sR0[2][a];
      dd += q * q;
    }
    out->d_nm = sqrt(dd);
  }
}

// one thread per field: Eq. HB and the exchange in the qubit frames
__global__ void st_model_kernel(const hkp_gmatrix_result* __restrict__ gm,
                                const double* __restrict__ Jp, double n0, double n1, double n2,
                                double lambda, double d_in, int nB, const double* __restrict__ Bv,
                                hkp_st_point* __restrict__ pts, double2* __restrict__ Hout) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nB) return;
  const double n[3] = {n0, n1, n2};
  const double B[3] = {Bv[3 * k], Bv[3 * k + 1], Bv[3 * k + 2]};
  double gL[3][3], gR[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      gL[i][j] = gm->g_sym[2][i][j];
      gR[i][j] = gm->g_sym[3][i][j];
    }
  const double t = gm->t_eV, J = *Jp;
  const double theta = (d_in > 0.0 ? d_in : gm->d_nm) / lambda;
  double Rm[3][3], Rp[3][3], gLB[3], gRB[3], a[3], b[3];
  rotation(n, -theta, Rm);
  rotation(n, theta, Rp);
  matvec3(gL, B, gLB);
  matvec3(gR, B, gRB);
  matvec3(Rm, gLB, a);
  matvec3(Rp, gRB, b);
  hkp_st_point& P = pts[k];
  double bb[3], db[3];
  for (int i = 0; i < 3; ++i) {
    bb[i] = 0.5 * kMuB * (a[i] + b[i]);
    db[i] = 0.5 * kMuB * (a[i] - b[i]);
    P.bbar_eV[i] = bb[i];
    P.dbar_eV[i] = db[i];
  }
  P.dEz_eV = sqrt(db[0] * db[0] + db[1] * db[1] + db[2] * db[2]);
  // Eq. HB in the basis S(0,2), S(1,1), T+, T-, T0
  const double r2 = sqrt(2.0);
  double2 H[5][5];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) H[i][j] = make_double2(0.0, 0.0);
  H[0][0] = make_double2(2.0 * t * t / J, 0.0);
  H[0][1] = make_double2(r2 * t, 0.0);
  H[1][2] = make_double2(-db[0] / r2, -db[1] / r2);
  H[1][3] = make_double2(db[0] / r2, -db[1] / r2);
  H[1][4] = make_double2(db[2], 0.0);
  H[2][2] = make_double2(bb[2], 0.0);
  H[3][3] = make_double2(-bb[2], 0.0);
  H[2][4] = make_double2(bb[0] / r2, -bb[1] / r2);
  H[3][4] = make_double2(bb[0] / r2, bb[1] / r2);
  const int up[5][2] = {{0, 1}, {1, 2}, {1, 3}, {1, 4}, {2, 4}};
  for (int q = 0; q < 5; ++q) H[up[q][1]][up[q][0]] = cconj(H[up[q][0]][up[q][1]]);
  H[4][3] = cconj(H[3][4]);
  if (Hout)
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) Hout[(long long)k * 25 + i * 5 + j] = H[i][j];
  double2 V[5][5];
  double w[5];
  jacobi_herm<5>(H, V, w);
  for (int i = 0; i < 5; ++i) P.E_eV[i] = w[i];
  // J_hat = J R(-2 theta); J~ = R_L J_hat R_R^T
  double R2[3][3], RL[3][3], RR[3][3], T[3][3];
  rotation(n, -2.0 * theta, R2);
  qubit_frame(gLB, RL);
  qubit_frame(gRB, RR);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int m = 0; m < 3; ++m) s += J * R2[i][m] * RR[j][m];
      T[i][j] = s;   // J_hat R_R^T
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int m = 0; m < 3; ++m) s += RL[i][m] * T[m][j];
      P.Jtilde_eV[i][j] = s;
    }
  P.J_perp_eV = 0.5 * hypot(P.Jtilde_eV[0][0] + P.Jtilde_eV[1][1],
                            P.Jtilde_eV[0][1] - P.Jtilde_eV[1][0]);
  P.J_par_eV = P.Jtilde_eV[2][2];
}

unsigned blocks(long long n) { return (unsigned)((n + kT - 1) / kT); }

}  // namespace

hipError_t launch_position_weight(int nx, int ny, int nz, double h, double* buf, hipStream_t s) {
  const long long N = (long long)nx * ny * nz;
  position_weight_kernel<<<dim3(blocks(N), 4), kT, 0, s>>>(nx, ny, nz, h,
                                                           reinterpret_cast<double2*>(buf));
  return hipGetLastError();
}

hipError_t launch_zeeman_derivative(long long N, double kappa, double* buf, hipStream_t s) {
  zeeman_derivative_kernel<<<dim3(blocks(N), 4), kT, 0, s>>>(
      N, kMuB * (3.0 * kappa - 1.0), reinterpret_cast<double2*>(buf));
  return hipGetLastError();
}

hipError_t launch_gmatrix_post(const double* G, void* out, hipStream_t s) {
  gmatrix_post_kernel<<<1, 64, 0, s>>>(reinterpret_cast<const double2*>(G),
                                       static_cast<hkp_gmatrix_result*>(out));
  return hipGetLastError();
}

hipError_t launch_st_model(const void* gm, const double* J, const double n_so[3], double lambda,
                           double d, int nB, const double* B, void* pts, void* H, hipStream_t s) {
  st_model_kernel<<<(nB + 63) / 64, 64, 0, s>>>(
      static_cast<const hkp_gmatrix_result*>(gm), J, n_so[0], n_so[1], n_so[2], lambda, d, nB, B,
      static_cast<hkp_st_point*>(pts), static_cast<double2*>(H));
  return hipGetLastError();
}

}  // namespace hkp
