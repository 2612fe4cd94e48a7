// Autotuner for the stencil (Chebyshev step) kernel: times the tile shapes on
// the caller's grid and block size with HIP events and caches the fastest per
// (shape, nb, precision, stencil variant) for the life of the process; the
// variant is strain on/off and the link-phase kind (none, Bz = 0, general).
// A launch whose own variant was never tuned takes the shape tuned for
// another variant of the same shape, nb and precision, else the default.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "hkp_internal.h"
#include "solver.h"

namespace hkp {

StencilTune autotuned_shape(const hkp_grid& g, int nb, bool mixed, int variant);

namespace {

using Key = std::tuple<int, int, int, int, int>;   // nx, ny, nz, nb|nev, mixed
using TuneKey = std::tuple<int, int, int, int, int, int>;   // ... + variant
std::mutex g_mu;
std::map<TuneKey, StencilTune> g_cache;

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// HKP_STENCIL="tile_y,vgroup,dma[,zsplit]" forces one launch shape (tests of a variant);
// HKP_STENCIL2="tile_x,tile_y" the two-step kernel's tile ("0,0": one step per pass)
bool forced(StencilTune* t) {
  const char* e = std::getenv("HKP_STENCIL");
  if (!e || !e[0]) return false;
  StencilTune f;
  const int n = std::sscanf(e, "%d,%d,%d,%d", &f.tile_y, &f.vgroup, &f.dma, &f.zsplit);
  if (n < 3) return false;
  *t = f;
  return true;
}
void forced2(StencilTune* t) {
  const char* e = std::getenv("HKP_STENCIL2");
  if (!e || !e[0]) return;
  int tx = 0, ty = 0;
  if (std::sscanf(e, "%d,%d", &tx, &ty) == 2) {
    t->t2x = tx;
    t->t2y = ty;
  }
}

// block size per (nx, ny, nz, nev, mixed), set by hkp_autotune_block
std::map<Key, int> g_nb_cache;

}  // namespace

int block_size(const hkp_grid& g, const hkp_opts& o) {
  if (o.nb > 0) return o.nb;
  const long long n6 = 6LL * g.nx * g.ny * g.nz;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_nb_cache.find(
        Key{g.nx, g.ny, g.nz, o.nev, o.precision == HKP_PREC_MIXED ? 1 : 0});
    if (it != g_nb_cache.end()) return it->second;
  }
  return default_nb(o.nev, n6);
}

// Block size by measurement: one complete solve of the given Hamiltonian per
// candidate (eager, outputs discarded), wall time to convergence; the fastest
// converged candidate is cached for this grid, nev and precision.
int run_autotune_block(const hkp_grid& g, const hkp_material& mat, const hkp_opts& o,
                       const double* V, const double* strain, const double B[3],
                       const int* cand, int ncand, void* ws, size_t ws_bytes, void* stream,
                       int* nb_out, double* seconds_out) {
  int best = 0;
  double best_s = 1e300;
  const char* dbg = std::getenv("HKP_TUNE_TRACE");
  for (int k = 0; k < ncand; ++k) {
    hkp_opts oc = o;
    oc.nb = cand[k];
    oc.flags &= ~(HKP_FLAG_GRAPH | HKP_FLAG_X0);
    SolveArgs a{};
    a.plan = make_plan(g, oc, 1);
    if (plan_bytes(a.plan) > ws_bytes) {
      set_error("hkp_autotune_block: workspace too small for block size " +
                std::to_string(cand[k]));
      return HKP_E_WORKSPACE;
    }
    a.mat = mat;
    a.V = V;
    a.strain = strain;
    for (int i = 0; i < 3; ++i) a.B[i] = B[i];
    a.workspace = ws;
    a.stream = stream;
    a.tol = oc.tol_eV;
    a.max_iter = oc.max_iter;
    a.flags = oc.flags;
    a.seed = oc.seed;
    a.st = autotuned(g, oc.nb, oc.precision == HKP_PREC_MIXED, stencil_variant(strain != nullptr, B));
    a.graph_chunk = 4;
    const auto t0 = std::chrono::steady_clock::now();
    const int rc = run_solve(a, nullptr);
    const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rc < 0) return rc;
    const double sc = rc == HKP_OK ? s : 1e300;   // a candidate that did not converge loses
    if (seconds_out) seconds_out[k] = rc == HKP_OK ? s : -s;
    if (dbg && dbg[0] == '1') std::fprintf(stderr, "[hkp tune] nb %d: %.4f s (status %d)\n", cand[k], s, rc);
    if (sc < best_s) {
      best_s = sc;
      best = cand[k];
    }
  }
  if (best == 0) {
    set_error("hkp_autotune_block: no candidate converged within max_iter");
    return HKP_W_NOT_CONVERGED;
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_nb_cache[Key{g.nx, g.ny, g.nz, o.nev, o.precision == HKP_PREC_MIXED ? 1 : 0}] = best;
  }
  *nb_out = best;
  return HKP_OK;
}

int stencil_variant(bool strain, const double B[3]) {
  const int ph = (B[0] == 0.0 && B[1] == 0.0 && B[2] == 0.0) ? 0 : (B[2] != 0.0 ? 2 : 1);
  return (strain ? 1 : 0) | (ph << 1);
}

StencilTune autotuned(const hkp_grid& g, int nb, bool mixed, int variant) {
  StencilTune t = autotuned_shape(g, nb, mixed, variant);
  forced2(&t);
  return t;
}

// ---- the caches in a file, keyed by the device architecture
namespace {
std::string current_arch() {
  int n = 0, dev = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1 || hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return "none";
  }
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "none";
  }
  std::string a = p.gcnArchName;
  return a.empty() ? "none" : a;
}
}  // namespace

int tune_cache_save(const char* path) {
  if (!path) {
    set_error("hkp_tune_cache_save: NULL path");
    return HKP_E_ARG;
  }
  std::ostringstream o;
  o << "# hkp autotune cache 1\n";
  o << "arch " << current_arch() << "\n";
  int n = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto& kv : g_cache) {
      const auto& k = kv.first;
      const StencilTune& t = kv.second;
      o << "stencil " << std::get<0>(k) << ' ' << std::get<1>(k) << ' ' << std::get<2>(k) << ' '
        << std::get<3>(k) << ' ' << std::get<4>(k) << ' ' << std::get<5>(k) << ' ' << t.tile_y
        << ' ' << t.vgroup << ' ' << t.dma << ' ' << t.zsplit << ' ' << t.t2x << ' ' << t.t2y
        << "\n";
      ++n;
    }
    for (const auto& kv : g_nb_cache) {
      const auto& k = kv.first;
      o << "block " << std::get<0>(k) << ' ' << std::get<1>(k) << ' ' << std::get<2>(k) << ' '
        << std::get<3>(k) << ' ' << std::get<4>(k) << ' ' << kv.second << "\n";
      ++n;
    }
  }
  std::ofstream f(path, std::ios::trunc);
  if (!f || !(f << o.str()) || !f.flush()) {
    set_error(std::string("hkp_tune_cache_save: cannot write ") + path);
    return HKP_E_ARG;
  }
  return n;
}

int tune_cache_load(const char* path) {
  if (!path) {
    set_error("hkp_tune_cache_load: NULL path");
    return HKP_E_ARG;
  }
  std::ifstream f(path);
  if (!f) {
    set_error(std::string("hkp_tune_cache_load: cannot read ") + path);
    return HKP_E_ARG;
  }
  // parse everything first: a malformed file changes nothing
  std::string arch;
  std::vector<std::pair<TuneKey, StencilTune>> sten;
  std::vector<std::pair<Key, int>> blocks;
  std::string line;
  int lineno = 0;
  auto bad = [&](const std::string& why) {
    set_error("hkp_tune_cache_load: " + std::string(path) + " line " + std::to_string(lineno) +
              ": " + why);
    return HKP_E_ARG;
  };
  while (std::getline(f, line)) {
    ++lineno;
    if (line.empty() || line[0] == '#') continue;
    std::istringstream is(line);
    std::string kind;
    is >> kind;
    if (kind == "arch") {
      if (!(is >> arch)) return bad("arch without a name");
    } else if (kind == "stencil") {
      int v[12];
      for (int& x : v)
        if (!(is >> x)) return bad("stencil entry needs 12 integers");
      StencilTune t;
      t.tile_y = v[6];
      t.vgroup = v[7];
      t.dma = v[8];
      t.zsplit = v[9];
      t.t2x = v[10];
      t.t2y = v[11];
      const bool ok = v[0] > 0 && v[1] > 0 && v[2] > 0 && v[3] >= 1 && v[3] <= HKP_NB_MAX &&
                      (v[4] == 0 || v[4] == 1) && v[5] >= 0 && v[5] < 6 &&
                      (t.tile_y == 1 || t.tile_y == 2 || t.tile_y == 4) && t.vgroup >= 1 &&
                      (t.dma == 0 || t.dma == 1) && t.zsplit >= 0 && t.zsplit <= 2 &&
                      t.t2x >= 0 && t.t2y >= 0;
      if (!ok) return bad("stencil entry out of range");
      sten.push_back({TuneKey{v[0], v[1], v[2], v[3], v[4], v[5]}, t});
    } else if (kind == "block") {
      int v[6];
      for (int& x : v)
        if (!(is >> x)) return bad("block entry needs 6 integers");
      if (v[0] < 1 || v[1] < 1 || v[2] < 1 || v[3] < 1 || (v[4] != 0 && v[4] != 1) ||
          v[5] <= v[3] || v[5] > HKP_NB_MAX)
        return bad("block entry out of range");
      blocks.push_back({Key{v[0], v[1], v[2], v[3], v[4]}, v[5]});
    } else {
      return bad("unknown entry '" + kind + "'");
    }
  }
  if (arch.empty()) {
    lineno = 0;
    return bad("no arch line");
  }
  if (arch != current_arch()) return 0;   // another device's choices
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto& e : sten) g_cache[e.first] = e.second;
  for (const auto& e : blocks) g_nb_cache[e.first] = e.second;
  return (int)(sten.size() + blocks.size());
}

void tune_cache_clear() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache.clear();
  g_nb_cache.clear();
}

bool two_step_tuned(const hkp_grid& g, int nb) {
  StencilTune f;
  forced2(&f);
  if (f.t2x > 0) return true;
  if (std::getenv("HKP_STENCIL2")) return false;   // forced off ("0,0")
  std::lock_guard<std::mutex> lk(g_mu);
  for (int v = 0; v < 6; ++v) {
    auto it = g_cache.find(TuneKey{g.nx, g.ny, g.nz, nb, 1, v});
    if (it != g_cache.end() && it->second.t2x > 0) return true;
  }
  return false;
}

StencilTune autotuned_shape(const hkp_grid& g, int nb, bool mixed, int variant) {
  StencilTune t;
  if (forced(&t)) return t;
  std::lock_guard<std::mutex> lk(g_mu);
  const int m = mixed ? 1 : 0;
  auto it = g_cache.find(TuneKey{g.nx, g.ny, g.nz, nb, m, variant});
  if (it != g_cache.end()) return it->second;
  for (int v = 0; v < 6; ++v) {
    it = g_cache.find(TuneKey{g.nx, g.ny, g.nz, nb, m, v});
    if (it != g_cache.end()) return it->second;
  }
  // untuned default (the fastest shape measured on the fin and double-dot
  // grids): two-row tiles, rows staged global -> LDS directly when tiles are
  // full along x
  t.tile_y = g.ny >= 2 ? 2 : 1;
  t.dma = g.nx % 64 == 0 ? 1 : 0;
  return t;
}

int run_autotune(const hkp_grid& g, int nb, bool mixed, bool strain, int field, void* ws,
                 size_t ws_bytes, void* stream, hkp_tune* out) {
  const long long N = (long long)g.nx * g.ny * g.nz, n6 = 6 * N;
  const size_t esz = mixed ? 8 : 16;
  size_t need = al(6 * N * 8) + al((size_t)g.nz * 16) + al((size_t)g.nz * g.nx * 16) +
                2 * al((size_t)nb * n6 * esz);
  if (ws_bytes < need) {
    set_error("autotune workspace too small: need " + std::to_string(need) + " bytes");
    return HKP_E_WORKSPACE;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* p = reinterpret_cast<char*>(ws);
  size_t off = 0;
  auto take = [&](size_t b) {
    char* q = p + off;
    off += al(b);
    return q;
  };
  void* D = take(6 * N * 8);
  void* wt = take((size_t)g.nz * 16);
  void* vt = take((size_t)g.nz * g.nx * 16);
  void* X = take((size_t)nb * n6 * esz);
  void* O = take((size_t)nb * n6 * esz);
  void* Y = O;   // the solver's filter writes over the block it reads as Y_old
  // contents do not affect the timing; give them finite values
  if (hipMemsetAsync(p, 0, off, s) != hipSuccess) return HKP_E_HIP;
  hkp_material m;
  hkp_default_material(&m);
  // field 1: B along x (link phases uniform over a z-plane); 2: B with a z
  // component (the general phase kernel)
  const double B[3] = {field ? 0.5 : 0.0, 0.0, field == 2 ? 0.5 : 0.0};
  const StencilConsts<double> c = make_consts(m, g.h_nm, B);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return HKP_E_HIP;
  StencilTune best;
  double best_us = 1e300;
  const char* dbg = std::getenv("HKP_TUNE_TRACE");
  std::vector<int> groups;   // 1 (vector-major), 2, 4, nb (tile-major)
  for (int vg : {1, 2, 4, nb})
    if (vg <= nb && std::find(groups.begin(), groups.end(), vg) == groups.end()) groups.push_back(vg);
  for (int dma = 0; dma < 2; ++dma)
  for (int vg : groups)
  for (int ty : {1, 2, 4}) {
    if (ty > 1 && ty > 2 * g.ny) continue;
    if (dma && g.nx % 64 != 0) continue;
    StencilLaunch a{};
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.nvec = nb;
    a.batch = 1;
    a.in = X;
    a.old = O;
    a.old_fp64 = !mixed;
    a.out = Y;
    a.out_fp64 = !mixed;
    a.D = D;
    a.strain = strain;
    a.wtab = field ? wt : nullptr;
    a.vtab = field ? vt : nullptr;
    a.phase_general = field == 2;
    a.coef.alpha = 1.0;
    a.coef.shift = 0.5;
    a.coef.beta = -1.0;
    a.tile_y = ty;
    a.vgroup = vg;
    a.dma = dma;
    a.fp64 = !mixed;
    if (launch_stencil(a, c, s) != hipSuccess) continue;   // warm-up
    const int reps = 5;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r) (void)launch_stencil(a, c, s);
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double us = 1e3 * ms / reps;
    if (dbg && dbg[0] == '1')
      std::fprintf(stderr, "[hkp tune] ty %d vgroup %d dma %d: %.1f us\n", ty, vg, dma, us);
    if (us < best_us) {
      best_us = us;
      best.tile_y = ty;
      best.vgroup = vg;
      best.dma = dma;
    }
  }
  // two-step passes (FP32 filter): faster than two one-step passes of the best shape?
  double best2_us = 0.0;
  if (mixed && field != 2 && two_step_grid(g.nx, 6)) {
    void* Y1 = take((size_t)nb * n6 * esz);
    void* Y2 = take((size_t)nb * n6 * esz);
    if (off <= ws_bytes) {
      if (hipMemsetAsync(Y1, 0, 2 * al((size_t)nb * n6 * esz), s) != hipSuccess) return HKP_E_HIP;
      double b2 = 2.0 * best_us;
      for (int tx : {16, 32})
      for (int ty : {8, 12}) {
        Stencil2Launch a{};
        a.nx = g.nx;
        a.ny = g.ny;
        a.nz = g.nz;
        a.nvec = nb;
        a.batch = 1;
        a.in = X;
        a.old = O;
        a.out1 = Y1;
        a.out2 = Y2;
        a.D = D;
        a.strain = strain;
        a.zero = X;   // the timing blocks are all zero
        a.wtab = field ? wt : nullptr;
        a.vtab = field ? vt : nullptr;
        a.host1[0] = a.host2[0] = 1.0;
        a.host1[1] = a.host2[1] = 0.5;
        a.host1[2] = a.host2[2] = -1.0;
        a.tile_x = tx;
        a.tile_y = ty;
        a.vgroup = best.vgroup;
        if (!stencil2_supported(a)) continue;
        if (launch_stencil2(a, c, s) != hipSuccess) continue;   // warm-up
        const int reps = 5;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r) (void)launch_stencil2(a, c, s);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double us = 1e3 * ms / reps;
        if (dbg && dbg[0] == '1')
          std::fprintf(stderr, "[hkp tune] two-step %d x %d: %.1f us (one-step pair %.1f us)\n",
                       tx, ty, us, 2.0 * best_us);
        if (us < b2) {
          b2 = us;
          best.t2x = tx;
          best.t2y = ty;
          best2_us = us;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[TuneKey{g.nx, g.ny, g.nz, nb, mixed ? 1 : 0, stencil_variant(strain, B)}] = best;
  }
  out->tile_y = best.tile_y;
  out->vgroup = best.vgroup;
  out->dma = best.dma;
  out->two_step_tx = best.t2x;
  out->two_step_ty = best.t2y;
  out->reserved = 0;
  out->us_per_step_two = best2_us > 0 ? best2_us / 2.0 : 0.0;
  out->us_per_step = best_us;
  // algorithmic bytes of one filter step: read X and Y_old, write Y, plus fields
  const double bytes = 3.0 * nb * n6 * esz + (double)N * (mixed ? 28 : 56);
  out->gbps = bytes / (best_us * 1e-6) / 1e9;
  return HKP_OK;
}

}  // namespace hkp
