// Spin-free single-particle basis (paper Eq. H0, Sec. II.D) and its spin-orbit
// matrix (Eq. H1, Fig. 2d-e).
//
// Without spin-orbit coupling and magnetic field the |L S> Hamiltonian is two
// identical, uncoupled 3 x 3 orbital blocks.  A spin-free solve works on
// three-component vectors (internal [v][c][z][y][x], c = X, Y, Z of one spin):
// the stencil's spin-free variant touches half the bytes of a spinor, and the
// block kernels (Gram, rotation, residuals) see vectors of 3N entries.  Each
// orbital level appears once.  The orbital vectors cross the boundary as
// complex [v][x][y][z][3], no basis change and no gauge (B = 0).
//
// The spin-orbit matrix of M orbitals is formed from their 3M x 3M component
// overlaps <phi_i,b | phi_j,c> (the FP64 MFMA Gram kernel on the components
// gathered into 3M vectors) and the constant on-site operator
// (Delta_0 / 3)(1 - sum_a sigma_a (x) L_a), (L_a)_bc = -i eps_abc.
#include <hip/hip_runtime.h>

#include "hkp_internal.h"

namespace hkp {

namespace {

// [v][x][y][z][3] -> internal [v][c][z][y][x], c < 3
__global__ void orbital_to_internal_kernel(int nx, int ny, int nz, const double2* orb,
                                           double2* internal) {
  const long long N = (long long)nx * ny * nz;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (p >= N) return;
  const int x = (int)(p % nx);
  const int y = (int)((p / nx) % ny);
  const int z = (int)(p / ((long long)nx * ny));
  const long long a = ((long long)x * ny + y) * nz + z;
  const double2* src = orb + ((long long)v * N + a) * 3;
  double2* dst = internal + (long long)v * 3 * N + p;
  for (int c = 0; c < 3; ++c) dst[(long long)c * N] = src[c];
}

// internal [b][v][c][z][y][x] -> [b][v][x][y][z][3]
__global__ void internal_to_orbital_kernel(int nx, int ny, int nz, const double2* internal,
                                           long long in_bstride, double2* orb,
                                           long long out_bstride) {
  const long long N = (long long)nx * ny * nz;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y, b = blockIdx.z;
  if (p >= N) return;
  const int x = (int)(p % nx);
  const int y = (int)((p / nx) % ny);
  const int z = (int)(p / ((long long)nx * ny));
  const long long a = ((long long)x * ny + y) * nz + z;
  const double2* src = internal + (long long)b * in_bstride + (long long)v * 3 * N + p;
  double2* dst = orb + (long long)b * out_bstride + ((long long)v * N + a) * 3;
  for (int c = 0; c < 3; ++c) dst[c] = src[(long long)c * N];
}

// [M][N][3] -> [3M][N]: vector 3 i + b holds component b of orbital i
__global__ void gather_components_kernel(long long N, const double2* orb, double2* comp) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (p >= N) return;
  const double2* src = orb + ((long long)i * N + p) * 3;
  for (int b = 0; b < 3; ++b) comp[((long long)3 * i + b) * N + p] = src[b];
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 cmul2(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// H_SO[(s, b), (t, c)] = (d/3) (delta_st delta_bc - sum_a sigma_a[s][t] (L_a)[b][c])
__device__ double2 hso(int s, int b, int t, int c, double d3) {
  // sigma_x = [[0,1],[1,0]], sigma_y = [[0,-i],[i,0]], sigma_z = [[1,0],[0,-1]]
  const double2 sig[3][2][2] = {
      {{{0, 0}, {1, 0}}, {{1, 0}, {0, 0}}},
      {{{0, 0}, {0, -1}}, {{0, 1}, {0, 0}}},
      {{{1, 0}, {0, 0}}, {{0, 0}, {-1, 0}}}};
  double2 acc = make_double2((s == t && b == c) ? 1.0 : 0.0, 0.0);
  for (int a = 0; a < 3; ++a) {
    // (L_a)_bc = -i eps_abc
    double e = 0.0;
    if (a != b && b != c && a != c) e = ((b - a + 3) % 3 == 1) ? 1.0 : -1.0;
    if (e == 0.0) continue;
    const double2 L = make_double2(0.0, -e);
    const double2 t2 = cmul2(sig[a][s][t], L);
    acc.x -= t2.x;
    acc.y -= t2.y;
  }
  return make_double2(d3 * acc.x, d3 * acc.y);
}

// out[2i+s][2j+t] = delta_ij delta_st E_i + sum_bc O[3i+b][3j+c] H_SO[(s,b),(t,c)]
__global__ void soi_assemble_kernel(int M, const double2* O, const double* E, double d3,
                                    double2* out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = 2 * M;
  if (idx >= n * n) return;
  const int r = idx / n, q = idx % n;
  const int i = r >> 1, s = r & 1, j = q >> 1, t = q & 1;
  double2 acc = make_double2(0.0, 0.0);
  for (int b = 0; b < 3; ++b)
    for (int c = 0; c < 3; ++c)
      acc = cadd(acc, cmul2(O[(long long)(3 * i + b) * (3 * M) + 3 * j + c], hso(s, b, t, c, d3)));
  if (E && i == j && s == t) acc.x += E[i];
  out[idx] = acc;
}

unsigned blocks(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_orbital_to_internal(int nx, int ny, int nz, int nvec, const void* orb,
                                      double* internal, hipStream_t s) {
  const long long N = (long long)nx * ny * nz;
  constexpr int kChunk = 32768;   // grid y extent within the launch limit
  for (int v0 = 0; v0 < nvec; v0 += kChunk) {
    const int nv = nvec - v0 < kChunk ? nvec - v0 : kChunk;
    orbital_to_internal_kernel<<<dim3(blocks(N), (unsigned)nv), 256, 0, s>>>(
        nx, ny, nz, static_cast<const double2*>(orb) + (long long)v0 * N * 3,
        reinterpret_cast<double2*>(internal) + (long long)v0 * N * 3);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_internal_to_orbital(int nx, int ny, int nz, int nvec, int batch,
                                      const double* internal, long long in_bstride, void* orb,
                                      long long out_bstride, hipStream_t s) {
  const long long N = (long long)nx * ny * nz;
  internal_to_orbital_kernel<<<dim3(blocks(N), (unsigned)nvec, (unsigned)batch), 256, 0, s>>>(
      nx, ny, nz, reinterpret_cast<const double2*>(internal), in_bstride,
      static_cast<double2*>(orb), out_bstride);
  return hipGetLastError();
}

hipError_t launch_gather_components(long long N, int M, const void* orb, double* comp,
                                    hipStream_t s) {
  gather_components_kernel<<<dim3(blocks(N), (unsigned)M), 256, 0, s>>>(
      N, static_cast<const double2*>(orb), reinterpret_cast<double2*>(comp));
  return hipGetLastError();
}

hipError_t launch_soi_assemble(int M, const double* O, const double* E, double delta_so,
                               void* out, hipStream_t s) {
  const int n = 2 * M;
  soi_assemble_kernel<<<blocks((long long)n * n), 256, 0, s>>>(
      M, reinterpret_cast<const double2*>(O), E, delta_so / 3.0, static_cast<double2*>(out));
  return hipGetLastError();
}

}  // namespace hkp
