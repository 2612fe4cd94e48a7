// Field setup, boundary transforms, the gate -> potential map and the
// Hellmann-Feynman gradient.
#include <map>
#include <mutex>

#include "hkp_internal.h"

// Block partial sums of the allocation-free Hellmann-Feynman gradient: one
// value per (workgroup, gate) of the gradient kernel, 1024 x 16 doubles
// (128 KiB), held on every device the library runs on until the process ends.
// Host code never passes this name to a kernel: it takes the device address
// from hkp::hf_scratch (hipGetSymbolAddress, once per device).
static __device__ __align__(256) double scratch[1024 * 16];

namespace hkp {

namespace {

constexpr double kS3 = 1.7320508075688772935;
constexpr double kS2 = 1.4142135623730950488;
constexpr double kInvS6 = 0.40824829046386301637;

// psi_J = U psi_LS at every grid point.  Rows: |J m_j> (|3/2,+3/2>, |3/2,+1/2>,
// |3/2,-1/2>, |3/2,-3/2>, |1/2,+1/2>, |1/2,-1/2>), columns: |X up>, |Y up>,
// |Z up>, |X dn>, |Y dn>, |Z dn>; every entry times 1/sqrt(6).  These are the
// standard p-orbital expansions of the |J m_j> states, e.g.
// |3/2,+3/2> = -(i/sqrt2) (X + iY) up, in the phase convention in which the
// |J m_j> Hamiltonian takes the Luttinger-Kohn layout of Eq. LK.
__constant__ double kUre[6][6] = {
    {0, kS3, 0, 0, 0, 0},
    {0, 0, 0, 0, 1, 0},
    {0, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, kS3, 0},
    {0, 0, 0, 0, -kS2, 0},
    {0, kS2, 0, 0, 0, 0}};
__constant__ double kUim[6][6] = {
    {kS3, 0, 0, 0, 0, 0},
    {0, 0, -2, 1, 0, 0},
    {-1, 0, 0, 0, 0, -2},
    {0, 0, 0, -kS3, 0, 0},
    {0, 0, -kS2, -kS2, 0, 0},
    {-kS2, 0, 0, 0, 0, kS2}};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// gauge function chi (coordinates about the box centre)
__device__ __forceinline__ double chi_at(int i, int j, int k, int nx, int ny, int nz, double h,
                                         double Bx, double By, double Bz) {
  const double X = (i - 0.5 * (nx - 1)) * h, Y = (j - 0.5 * (ny - 1)) * h,
               Z = (k - 0.5 * (nz - 1)) * h;
  return -0.5 * Bz * X * Y - 0.5 * By * X * Z + 0.5 * Bx * Y * Z;
}

__global__ void onsite_kernel(int nx, int ny, int nz, const double* V, long long V_bstride,
                              const double* strain, double l_, double m_, double n_,
                              double* D64, float* D32, long long D_bstride, int with_strain) {
  const long long N = (long long)nx * ny * nz;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (p >= N) return;
  // internal index p = (z ny + y) nx + x
  const int x = (int)(p % nx);
  const int y = (int)((p / nx) % ny);
  const int z = (int)(p / ((long long)nx * ny));
  const long long a = ((long long)x * ny + y) * nz + z;  // ABI index
  const double v = V[(long long)b * V_bstride + a];
  double d[6];
  if (with_strain) {
    const double* e = strain + 6 * a;
    const double tr = e[0] + e[1] + e[2];
    d[0] = v + l_ * e[0] + m_ * (tr - e[0]);
    d[1] = v + l_ * e[1] + m_ * (tr - e[1]);
    d[2] = v + l_ * e[2] + m_ * (tr - e[2]);
    d[3] = n_ * e[3];  // yz
    d[4] = n_ * e[4];  // xz
    d[5] = n_ * e[5];  // xy
  } else {
    d[0] = v;
  }
  const int nd = with_strain ? 6 : 1;
  double* o64 = D64 + (long long)b * D_bstride;
  for (int c = 0; c < nd; ++c) o64[c * N + p] = d[c];
  if (D32) {
    float* o32 = D32 + (long long)b * D_bstride;
    for (int c = 0; c < nd; ++c) o32[c * N + p] = (float)d[c];
  }
}

__global__ void phase_kernel(int nx, int nz, double h, double Bx, double By, double Bz,
                             double* w64, double* v64, float* w32, float* v32) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const double kh = kEoverHbar * h;
  if (t < nz) {
    const double Z = (t - 0.5 * (nz - 1)) * h;
    double s, c;
    sincos(kh * By * Z, &s, &c);
    w64[2 * t] = c;
    w64[2 * t + 1] = s;
    if (w32) {
      w32[2 * t] = (float)c;
      w32[2 * t + 1] = (float)s;
    }
  }
  if (t < nx * nz) {
    const int x = t % nx, z = t / nx;
    const double X = (x - 0.5 * (nx - 1)) * h, Z = (z - 0.5 * (nz - 1)) * h;
    double s, c;
    sincos(kh * (Bz * X - Bx * Z), &s, &c);
    v64[2 * t] = c;
    v64[2 * t + 1] = s;
    if (v32) {
      v32[2 * t] = (float)c;
      v32[2 * t + 1] = (float)s;
    }
  }
}

// The two layouts of a block run along different axes: the ABI's [v][x][y][z][6]
// has z (then the six components) fastest, the internal [v][c][z][y][x] has x
// fastest.  A workgroup converts a 16 x 16 tile of (x, z) points of one y row of
// one vector through LDS: it reads the side whose fast axis it can cover with
// consecutive lanes (16 points of one row), transforms, and writes the other side
// the same way (for the ABI, 16 z points x 6 components = 1.5 KiB contiguous per x).
constexpr int kTile = 16;
constexpr int kTileRow = kTile * 6 + 1;   // complex entries per x row of the tile (padded)

struct TileCoord {
  int x0, y, z0;
};
__device__ __forceinline__ TileCoord tile_coord(int nx, int ny, int nz) {
  const int ntx = (nx + kTile - 1) / kTile;
  int t = blockIdx.x;
  TileCoord c;
  c.x0 = (t % ntx) * kTile;
  t /= ntx;
  c.y = t % ny;
  c.z0 = (t / ny) * kTile;
  return c;
}

// ABI block (J, symmetric gauge) -> internal (LS, GPU gauge)
template <typename TO>
__global__ void __launch_bounds__(256)
abi_to_internal_kernel(int nx, int ny, int nz, double h, double Bx, double By, double Bz,
                       const double2* abi, TO* internal) {
  __shared__ double2 tile[kTile][kTileRow];   // [x][z * 6 + c]
  const long long N = (long long)nx * ny * nz;
  const int v = blockIdx.y;
  const TileCoord tc = tile_coord(nx, ny, nz);
  {
    // read: lanes along z (and the six components), one x per 16 lanes
    const int xo = threadIdx.x >> 4, zo = threadIdx.x & 15;
    const int x = tc.x0 + xo, z = tc.z0 + zo;
    if (x < nx && z < nz) {
      const long long a = ((long long)x * ny + tc.y) * nz + z;
      const double2* src = abi + ((long long)v * N + a) * 6;
      double2 j[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) j[c] = src[c];
      double s, co;
      sincos(kEoverHbar * chi_at(x, tc.y, z, nx, ny, nz, h, Bx, By, Bz), &s, &co);
      const double2 g = make_double2(co, s);  // exp(+i k chi)
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        // (U^H psi_J)_c = sum_j conj(U_jc) psi_J,j
        double2 acc = make_double2(0, 0);
#pragma unroll
        for (int r = 0; r < 6; ++r) {
          const double2 u = make_double2(kUre[r][c] * kInvS6, -kUim[r][c] * kInvS6);
          const double2 t = cmul(u, j[r]);
          acc.x += t.x;
          acc.y += t.y;
        }
        tile[xo][zo * 6 + c] = cmul(g, acc);
      }
    }
  }
  __syncthreads();
  {
    // write: lanes along x
    const int xi = threadIdx.x & 15, zi = threadIdx.x >> 4;
    const int x = tc.x0 + xi, z = tc.z0 + zi;
    if (x < nx && z < nz) {
      const long long p = ((long long)z * ny + tc.y) * nx + x;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const double2 w = tile[xi][zi * 6 + c];
        TO* dst = internal + 2 * (((long long)v * 6 + c) * N + p);
        dst[0] = (TO)w.x;
        dst[1] = (TO)w.y;
      }
    }
  }
}

// internal (LS, GPU gauge) -> ABI block (J, symmetric gauge); vector v of batch
// member b
__global__ void __launch_bounds__(256)
internal_to_abi_kernel(int nx, int ny, int nz, double h, double Bx, double By, double Bz,
                       const double2* internal, long long in_bstride, double2* abi,
                       long long abi_bstride, int nvec) {
  __shared__ double2 tile[kTile][kTileRow];   // [x][z * 6 + r]
  const long long N = (long long)nx * ny * nz;
  const int v = blockIdx.y;
  const int b = blockIdx.z;
  const TileCoord tc = tile_coord(nx, ny, nz);
  {
    // read: lanes along x
    const int xi = threadIdx.x & 15, zi = threadIdx.x >> 4;
    const int x = tc.x0 + xi, z = tc.z0 + zi;
    if (x < nx && z < nz) {
      const long long p = ((long long)z * ny + tc.y) * nx + x;
      const double2* src = internal + (long long)b * in_bstride + (long long)v * 6 * N;
      double2 l[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) l[c] = src[(long long)c * N + p];
      double s, co;
      sincos(kEoverHbar * chi_at(x, tc.y, z, nx, ny, nz, h, Bx, By, Bz), &s, &co);
      const double2 g = make_double2(co, -s);  // exp(-i k chi)
#pragma unroll
      for (int c = 0; c < 6; ++c) l[c] = cmul(g, l[c]);
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        double2 acc = make_double2(0, 0);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const double2 u = make_double2(kUre[r][c] * kInvS6, kUim[r][c] * kInvS6);
          const double2 t = cmul(u, l[c]);
          acc.x += t.x;
          acc.y += t.y;
        }
        tile[xi][zi * 6 + r] = acc;
      }
    }
  }
  __syncthreads();
  {
    // write: lanes along z (16 points x 6 components contiguous per x)
    const int xo = threadIdx.x >> 4, zo = threadIdx.x & 15;
    const int x = tc.x0 + xo, z = tc.z0 + zo;
    if (x < nx && z < nz) {
      const long long a = ((long long)x * ny + tc.y) * nz + z;
      double2* dst = abi + (long long)b * abi_bstride + ((long long)v * N + a) * 6;
#pragma unroll
      for (int r = 0; r < 6; ++r) dst[r] = tile[xo][zo * 6 + r];
    }
  }
}

__global__ void gate_kernel(long long N, int G, const double* Vbg, const double* L,
                            const double* Vg, double* out) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  double v = Vbg[p];
  for (int g = 0; g < G; ++g) v = fma(Vg[g], L[(long long)g * N + p], v);
  out[p] = v;
}

constexpr int kHfThreads = 256;
constexpr int kHfMaxG = 16;

// grad partials: one value per (block, g).  Items are (state n, point p) pairs
// in state-major order, so consecutive threads read consecutive 96-byte
// spinors (one contiguous sweep of psi per state); each thread takes two items
// per loop trip with all their loads issued together.  p and n advance by the
// grid stride without divisions.
__global__ void __launch_bounds__(kHfThreads)
hf_partial_kernel(long long N, int nev, const double2* psi, const double* w, int G,
                  const double* L, double* partial) {
  double acc[kHfMaxG];
#pragma unroll
  for (int g = 0; g < kHfMaxG; ++g) acc[g] = 0.0;
  const long long total = (long long)nev * N;
  const long long stride = (long long)gridDim.x * blockDim.x;
  long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long n = j / N, p = j - n * N;
  auto advance = [&](long long& nn, long long& pp) {
    pp += stride;
    while (pp >= N) {
      pp -= N;
      ++nn;
    }
  };
  auto item = [&](long long jj, long long nn, long long pp) {
    const double2* q = psi + jj * 6;
    double2 v[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = q[c];
    double Lg[kHfMaxG];
#pragma unroll
    for (int g = 0; g < kHfMaxG; ++g) Lg[g] = g < G ? L[(long long)g * N + pp] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) s = fma(v[c].x, v[c].x, fma(v[c].y, v[c].y, s));
    const double ws = w[nn] * s;
#pragma unroll
    for (int g = 0; g < kHfMaxG; ++g)
      if (g < G) acc[g] = fma(ws, Lg[g], acc[g]);
  };
  for (; j + stride < total; j += 2 * stride) {
    long long n2 = n, p2 = p;
    advance(n2, p2);
    item(j, n, p);
    item(j + stride, n2, p2);
    n = n2;
    p = p2;
    advance(n, p);
  }
  if (j < total) item(j, n, p);
  __shared__ double red[kHfThreads / 64][kHfMaxG];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int g = 0; g < kHfMaxG; ++g) {
    if (g < G) {
      double v = acc[g];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0) red[wv][g] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < G) {
    double v = 0.0;
    for (int k = 0; k < kHfThreads / 64; ++k) v += red[k][threadIdx.x];
    partial[(long long)blockIdx.x * G + threadIdx.x] = v;
  }
}

// one workgroup per g: each thread sums a strided slice of the block partials,
// then waves and workgroup reduce in a fixed order (deterministic)
__global__ void __launch_bounds__(kHfThreads)
hf_reduce_kernel(int nblk, int G, const double* partial, double* grad) {
  const int g = blockIdx.x;
  double v = 0.0;
  for (int k = threadIdx.x; k < nblk; k += kHfThreads) v += partial[(long long)k * G + g];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __shared__ double red[kHfThreads / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < kHfThreads / 64; ++k) t += red[k];
    grad[g] = t;
  }
}

}  // namespace

hipError_t launch_onsite(const hkp_material& m, int nx, int ny, int nz, int batch,
                         const double* V, long long V_bstride, const double* strain,
                         double* D64, float* D32, long long D_bstride, hipStream_t s) {
  const long long N = (long long)nx * ny * nz;
  // Bir-Pikus orbital coefficients in the hole picture
  const double l_ = -(m.a_v_eV + 2.0 * m.b_eV);
  const double m_ = -(m.a_v_eV - m.b_eV);
  const double n_ = -kS3 * m.d_eV;
  dim3 grid((unsigned)((N + 255) / 256), (unsigned)batch);
  onsite_kernel<<<grid, 256, 0, s>>>(nx, ny, nz, V, V_bstride, strain, l_, m_, n_, D64, D32,
                                     D_bstride, strain != nullptr);
  return hipGetLastError();
}

hipError_t launch_phase_tables(int nx, int nz, double h, const double B[3], double* w64,
                               double* v64, float* w32, float* v32, hipStream_t s) {
  const int n = nx * nz > nz ? nx * nz : nz;
  phase_kernel<<<(n + 255) / 256, 256, 0, s>>>(nx, nz, h, B[0], B[1], B[2], w64, v64, w32, v32);
  return hipGetLastError();
}

namespace {
// workgroups of a layout conversion: 16 x 16 (x, z) tiles of every y row
unsigned conv_tiles(int nx, int ny, int nz) {
  return (unsigned)(((nx + kTile - 1) / kTile) * ny * ((nz + kTile - 1) / kTile));
}
}  // namespace

hipError_t launch_abi_to_internal(int nx, int ny, int nz, double h, const double B[3],
                                  int nvec, const void* abi, void* internal, int to_fp32,
                                  hipStream_t s) {
  const long long N = (long long)nx * ny * nz;
  // vectors in chunks: the grid's y extent stays within the launch limit
  constexpr int kChunk = 32768;
  for (int v0 = 0; v0 < nvec; v0 += kChunk) {
    const int nv = nvec - v0 < kChunk ? nvec - v0 : kChunk;
    const long long off = (long long)v0 * N * 6;   // complex entries before the chunk
    dim3 grid(conv_tiles(nx, ny, nz), (unsigned)nv);
    if (to_fp32)
      abi_to_internal_kernel<float><<<grid, 256, 0, s>>>(
          nx, ny, nz, h, B[0], B[1], B[2], (const double2*)abi + off,
          (float*)internal + 2 * off);
    else
      abi_to_internal_kernel<double><<<grid, 256, 0, s>>>(
          nx, ny, nz, h, B[0], B[1], B[2], (const double2*)abi + off,
          (double*)internal + 2 * off);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_internal_to_abi(int nx, int ny, int nz, double h, const double B[3],
                                  int nvec, int batch, const void* internal,
                                  long long in_bstride, void* abi, long long abi_bstride,
                                  hipStream_t s) {
  dim3 grid(conv_tiles(nx, ny, nz), (unsigned)nvec, (unsigned)batch);
  internal_to_abi_kernel<<<grid, 256, 0, s>>>(nx, ny, nz, h, B[0], B[1], B[2],
                                              (const double2*)internal, in_bstride,
                                              (double2*)abi, abi_bstride, nvec);
  return hipGetLastError();
}

hipError_t launch_gate_potential(long long N, int G, const double* Vbg, const double* L,
                                 const double* Vg, double* out, hipStream_t s) {
  gate_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(N, G, Vbg, L, Vg, out);
  return hipGetLastError();
}

int hf_blocks() { return 1024; }

size_t hf_partial_bytes(int G) { return (size_t)hf_blocks() * G * 8; }

size_t hf_scratch_bytes() { return sizeof(scratch); }

hipError_t hf_scratch(double** out) {
  static_assert(sizeof(scratch) == 1024 * kHfMaxG * sizeof(double),
                "scratch holds hf_blocks() x kHfMaxG partial sums");
  static std::mutex mu;
  static std::map<int, double*> ptr;   // device ordinal -> address of its copy
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  auto it = ptr.find(dev);
  if (it == ptr.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    it = ptr.emplace(dev, static_cast<double*>(p)).first;
  }
  *out = it->second;
  return hipSuccess;
}

hipError_t launch_hf_grad(long long N, int nev, const void* psi, const double* w, int G,
                          const double* L, double* partial, double* grad, hipStream_t s) {
  if (G > kHfMaxG) return hipErrorInvalidValue;
  const int nblk = hf_blocks();
  hf_partial_kernel<<<nblk, kHfThreads, 0, s>>>(N, nev, (const double2*)psi, w, G, L, partial);
  hf_reduce_kernel<<<G, kHfThreads, 0, s>>>(nblk, G, partial, grad);
  return hipGetLastError();
}

}  // namespace hkp
