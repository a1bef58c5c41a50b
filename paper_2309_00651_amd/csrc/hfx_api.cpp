// C ABI of the exact-exchange library: plan construction, argument
// validation, workspace layout and the launch sequence of each entry point.
//
// Pair work is scheduled in tile pairs of R rows x T columns (T = variant
// tile, R = rows per tile pair, a multiple of T).  Blocks of R orbitals meet
// in round-robin rounds (circle method); a block pair is cut into R / T tile
// pairs, one per column tile, and the tile pairs of one round with the same
// column tile share no orbital.  A batch is a slice of such a set, and its
// three pipeline passes run back to back on the caller's stream.  This makes
// K psi accumulation race-free and its order fixed (the pair loop of Eq. (vx)
// split over tiles, in the spirit of the paper's task groups, which also
// divide the pair list and sum the partial operators).
#include "../../include/hfx.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "hfx_internal.hpp"
#include "schedule.hpp"
#include "tune.hpp"
#include "twiddle.hpp"

using namespace hfx;

// Rows per tile pair when the plan options name none: 32 from 256 orbitals
// on, else 16 (measured on one MI355X over 64-512 orbitals and 64^3-128^3
// grids: never slower than 8 rows, within 2.5 % of the best choice).
int hfx::default_rows(int n_orb) { return n_orb >= 256 ? 32 : 16; }

namespace {

thread_local std::string g_last_error;

hfx_status fail(hfx_status s, const std::string& msg) {
  g_last_error = msg;
  hfx::log_line(std::string(hfx_status_string(s)) + ": " + msg);
  return s;
}

}  // namespace

void hfx::set_error(const std::string& msg) { g_last_error = msg; }

void hfx::log_line(const std::string& msg) {
  static const bool on = [] {
    const char* e = std::getenv("HFX_LOG");
    return e && *e && std::strcmp(e, "0") != 0;
  }();
  if (on) std::fprintf(stderr, "[hfx] %s\n", msg.c_str());
}

namespace {

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(e_ == hipErrorOutOfMemory ? HFX_ENOMEM : HFX_EDEVICE,            \
                  std::string(#expr) + ": " + hipGetErrorString(e_));              \
  } while (0)

struct SystemPlan {
  hfx_system sys;
  const Variant* var = nullptr;
  int n = 0;
  long long nr = 0;
  double dv = 0.0;
  int rows = 8;  // rows per tile pair (a multiple of the variant's tile)
  // band limit: pair densities vanish on kz planes |kz| > kz_max (>= nz / 2:
  // no plane is skipped)
  int kz_max = 1 << 30;
  int kx_max = 1 << 30;  // the same along x (from L_x)
  int ky_max = 1 << 30;  // and along y (from L_y)
  int tiles_per_batch = 1;
  int slots_per_batch = 0;
  std::vector<TileDesc> tiles;
  std::vector<int> active;
  std::vector<Batch> batches;
  long long n_partials = 0;
  // device tables (owned)
  void* vtab = nullptr;
  void* tw[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  TileDesc* d_tiles = nullptr;
  int* d_active = nullptr;
  void* d_zero = nullptr;  // kZeroBytes of zeros: what pruned kz planes read as (band-limited plans)
  // offsets inside the caller's workspace
  size_t off_psi32 = 0, off_grids = 0, off_partials = 0, off_gemm = 0, off_ortho = 0;
  // K psi staging of the gradient (float32 plans) and of hfx_exchange_matrix
  // (both precisions): n_orb x N_r values of the working precision
  size_t off_kpsi = 0;
  size_t off_mean = 0;  // float32 plans: pair-density means (n_orb x n_orb float64)
  double v0 = 0.0;      // v(G = 0)
  // batch streams: 2 = consecutive batches alternate between the call's
  // stream and an owned stream, each with its own pair-grid buffer
  int nstreams = 1;
  size_t grid_bytes = 0;  // one pair-grid buffer
  // virtual group (emulated shard) of the tile rounds: rounds r with
  // r % shards == shard; group 0 also adds the G = 0 energy
  int shard = 0, shards = 1;
  long long tiles_cap = 0;
  // pair screening (s-MTACE): orbital order of the tiles and the kept pairs
  // (n_orb x n_orb bytes, original orbital indices); null when unscreened
  int* d_perm = nullptr;
  unsigned char* d_keep = nullptr;
  hipStream_t bstream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_acc[2] = {nullptr, nullptr};
  // offsets inside concatenated user buffers
  long long psi_off = 0, m_off = 0;
  long long orb_off = 0;  // first orbital of this system (per-orbital arrays)
  bool tuned = false;     // kernel configuration taken from the tune cache
};

}  // namespace

struct ProfRec {
  int pass;
  hipEvent_t start, stop;
  double bytes, flops;
};

struct hfx_plan_t {
  int prec = 0;
  std::vector<SystemPlan> sys;
  size_t ws_bytes = 0;
  size_t apply_bytes = 0;  // leading workspace bytes the energy and K psi calls use
  int device = 0;
  bool prof = false;
  bool capturing = false;
  bool quiet = false;  // no profiling events (a call that must not create any)
  bool check = false;  // check the orbitals before each exchange call (option check=1)
  // systems of one size class share launches: 1 always, 0 never, -1 (the
  // default) for systems whose own launches are small (see size_classes)
  int group = -1;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  // multi-system plans: one side stream per system (default priority) and
  // fork/join events; capture stream for graphs
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  hipStream_t cap = nullptr;
  std::string desc;  // hfx_plan_describe's text
  // Graphs bake the device addresses of the schedule tables into their
  // kernel arguments.  While any graph of the plan is alive, tables that
  // hfx_screen replaces are kept here instead of freed, and released when
  // the last graph is destroyed (or with the plan).
  int live_graphs = 0;
  std::vector<void*> retired;
};

struct hfx_graph_t {
  hfx_plan plan = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

// First compiled variant for an n x n x nz grid (the default), or the one named.
const Variant* find_variant(int n, int nz, int prec, const std::string& name = "") {
  int count = 0;
  const Variant* v = prec == HFX_FP64 ? variants_f64(&count) : variants_f32(&count);
  for (int i = 0; i < count; ++i)
    if (v[i].n == n && v[i].nz == nz && (name.empty() || name == v[i].name)) return &v[i];
  return nullptr;
}

std::string parse_option_str(const char* opts, const char* key) {
  if (!opts) return "";
  const std::string s(opts), k = std::string(key) + "=";
  size_t p = 0;
  while (p < s.size()) {
    size_t e = s.find(';', p);
    if (e == std::string::npos) e = s.size();
    const std::string item = s.substr(p, e - p);
    if (item.compare(0, k.size(), k) == 0) return item.substr(k.size());
    p = e + 1;
  }
  return "";
}

// Whether an item "key=..." is present (its value may be empty).
bool has_option(const char* opts, const char* key) {
  if (!opts) return false;
  const std::string s(opts), k = std::string(key) + "=";
  size_t p = 0;
  while (p < s.size()) {
    size_t e = s.find(';', p);
    if (e == std::string::npos) e = s.size();
    if (s.compare(p, k.size(), k) == 0) return true;
    p = e + 1;
  }
  return false;
}

// Integer option: def when absent; false when present but not a whole
// non-negative decimal number.
bool parse_option(const char* opts, const char* key, long long def, long long* out) {
  *out = def;
  const std::string v = parse_option_str(opts, key);
  if (v.empty()) return opts == nullptr || std::string(opts).find(std::string(key) + "=") ==
                                               std::string::npos;
  char* end = nullptr;
  errno = 0;
  const long long x = std::strtoll(v.c_str(), &end, 10);
  if (end == v.c_str() || *end != '\0' || errno != 0 || x < 0) return false;
  *out = x;
  return true;
}

// Every key of the option string is one of the known ones.
bool options_known(const char* opts, std::string* bad) {
  if (!opts) return true;
  static const char* known[] = {"tiles", "maxws", "variant", "streams", "shard", "mix", "rows",
                                "ecut", "tune_cache", "check", "group"};
  const std::string s(opts);
  size_t p = 0;
  while (p < s.size()) {
    size_t e = s.find(';', p);
    if (e == std::string::npos) e = s.size();
    const std::string item = s.substr(p, e - p);
    p = e + 1;
    if (item.empty()) continue;
    const std::string key = item.substr(0, item.find('='));
    bool ok = item.find('=') != std::string::npos;
    if (ok) {
      ok = false;
      for (const char* k : known) ok = ok || key == k;
    }
    if (!ok) {
      *bad = item;
      return false;
    }
  }
  return true;
}

// Value of a per-system option for system i: "key=v" applies to every
// system, "key=v0,v1,..." gives one value per system (exactly n_sys of them).
// Empty when the key is absent; false when a list has the wrong length.
bool per_system_value(const std::string& v, int i, int n_sys, std::string* out) {
  out->clear();
  if (v.find(',') == std::string::npos) {
    *out = v;
    return true;
  }
  std::vector<std::string> items;
  size_t p = 0;
  while (true) {
    const size_t e = v.find(',', p);
    items.push_back(v.substr(p, e == std::string::npos ? std::string::npos : e - p));
    if (e == std::string::npos) break;
    p = e + 1;
  }
  if ((int)items.size() != n_sys) return false;
  *out = items[i];
  return true;
}

// Whole non-negative decimal number.
bool parse_count(const std::string& v, long long* out) {
  char* end = nullptr;
  errno = 0;
  const long long x = std::strtoll(v.c_str(), &end, 10);
  if (v.empty() || end == v.c_str() || *end != '\0' || errno != 0 || x < 0) return false;
  *out = x;
  return true;
}

// Workgroups of pass 3 (and of pass 1 on full planes) per tile pair: flat
// bricks of `brick` consecutive points of the n x n plane (the kernels assert
// that they tile it).
int bricks_per_tile(const Variant* v) {
  return v->n * v->n / v->brick;
}

// Whether the forward z transform of pair_fwd runs at half length: pair
// densities with |kz| <= kz_max are sampled exactly by the even z points when
// 2 kz_max + 1 <= nz / 2 (the same test as the kernels' launchers).
bool half_z(const Variant* v, int kz_max) {
  return v->nzh > 0 && v->nz % 2 == 0 && kz_max <= (v->nz / 2 - 1) / 2;
}

// Whether a system's plane pass takes half-height input (pass 1 on the even
// rows only): x band within the plane kernel's band columns and y band within
// a quarter of the grid (the same test as the kernels' launchers, over every
// system of a launch).
bool half_y(const Variant* v, int kx_max, int ky_max) {
  return v->hy && kx_max <= v->qb && ky_max <= (v->n / 2 - 1) / 2;
}

// Whether the half-height input is half-width too (pass 1 on the even x
// columns of the even rows, quarter planes): x band within a quarter of the
// grid as well.
bool half_x(const Variant* v, int kx_max, int ky_max) {
  return v->xd && half_y(v, kx_max, ky_max) && kx_max <= (v->n / 2 - 1) / 2;
}

ScheduleShape shape_of(const SystemPlan& sp) {
  ScheduleShape sh;
  sh.n_orb = sp.sys.n_orb;
  sh.tile = sp.var->tile;
  sh.rows = sp.rows;
  sh.bricks = bricks_per_tile(sp.var);
  sh.shard = sp.shard;
  sh.shards = sp.shards;
  return sh;
}

void take_schedule(SystemPlan& sp, Schedule&& s) {
  sp.tiles_per_batch = s.tiles_per_batch;
  sp.slots_per_batch = s.slots_per_batch;
  sp.tiles = std::move(s.tiles);
  sp.active = std::move(s.active);
  sp.batches = std::move(s.batches);
  sp.n_partials = s.n_partials;
}

// Unscreened schedule of a system (see schedule.hpp).
void schedule_all_pairs(SystemPlan& sp, long long tiles_cap) {
  take_schedule(sp, build_schedule(shape_of(sp), tiles_cap));
}

// Screened schedule: the batches fit the unscreened schedule's slots.
void schedule_kept_pairs(SystemPlan& sp, const std::vector<unsigned char>& keep,
                         const std::vector<int>& perm) {
  take_schedule(sp, build_screened_schedule(shape_of(sp), sp.slots_per_batch, keep, perm));
}

// v(G)/N_r on the FFT grid.  zero_dc: store 0 at G = 0 (float32 plans take the
// G = 0 term out of the transforms, see run_exchange).
template <typename T>
std::vector<T> kernel_table(const hfx_system& s, bool zero_dc, double scale) {
  const double pi = 3.14159265358979323846;
  const double om = s.L[0] * s.L[1] * s.L[2];
  const int nx = s.n[0], ny = s.n[1], nz = s.n[2];
  const double nr = (double)nx * ny * nz;
  const double rc = std::cbrt(3.0 * om / (4.0 * pi));
  std::vector<T> out((size_t)nx * ny * nz);
  auto freq = [](int k, int n) { return k < (n + 1) / 2 ? k : k - n; };
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const double gx = 2 * pi * freq(x, nx) / s.L[0];
        const double gy = 2 * pi * freq(y, ny) / s.L[1];
        const double gz = 2 * pi * freq(z, nz) / s.L[2];
        const double g2 = gx * gx + gy * gy + gz * gz;
        double v;
        if (s.kernel == HFX_KERNEL_TRUNCATED) {
          if (g2 == 0.0) {
            v = 2 * pi * rc * rc;
          } else {
            const double sh = std::sin(0.5 * std::sqrt(g2) * rc);
            v = 8 * pi * sh * sh / g2;
          }
        } else {
          const double w = s.param;
          v = g2 == 0.0 ? pi / (w * w) : -4 * pi * std::expm1(-g2 / (4 * w * w)) / g2;
        }
        out[((size_t)z * ny + y) * nx + x] = T(scale * v / nr);
      }
  if (zero_dc) out[0] = T(0);
  return out;
}

double kernel_g0(const hfx_system& s) {
  const double pi = 3.14159265358979323846;
  if (s.kernel == HFX_KERNEL_TRUNCATED) {
    const double rc = std::cbrt(3.0 * s.L[0] * s.L[1] * s.L[2] / (4.0 * pi));
    return 2 * pi * rc * rc;
  }
  return pi / (s.param * s.param);
}

template <typename T>
hfx_status upload(const std::vector<T>& h, void** d) {
  HIP_TRY(hipMalloc(d, std::max<size_t>(h.size(), 1) * sizeof(T)));
  if (!h.empty()) HIP_TRY(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return HFX_OK;
}

// float64 tables hold (re, im); float32 tables hold norm-optimised values
// (unit_f32 in twiddle.hpp).
hfx_status upload_twiddles(const int* r, int nr_, int prec, void** d) {
  const std::vector<double> t = twiddle_table(r, nr_);
  if (prec == HFX_FP64) return upload(t, d);
  std::vector<float> f(t.size());
  for (size_t i = 0; i < t.size(); i += 2) unit_f32(t[i], t[i + 1], &f[i], &f[i + 1]);
  return upload(f, d);
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

hfx_status validate_system(const hfx_system& s, int idx) {
  const std::string at = " (system " + std::to_string(idx) + ")";
  for (int k = 0; k < 3; ++k) {
    if (s.n[k] <= 0) return fail(HFX_EINVAL, "grid size must be positive" + at);
    if (!(s.L[k] > 0.0) || !std::isfinite(s.L[k]))
      return fail(HFX_EINVAL, "box length must be positive and finite" + at);
  }
  if (s.n_orb < 1) return fail(HFX_EINVAL, "n_orb must be >= 1" + at);
  if (s.kernel != HFX_KERNEL_TRUNCATED && s.kernel != HFX_KERNEL_ERFC)
    return fail(HFX_EINVAL, "unknown kernel" + at);
  if (s.kernel == HFX_KERNEL_ERFC && !(s.param > 0.0 && std::isfinite(s.param)))
    return fail(HFX_EINVAL, "erfc kernel needs w > 0" + at);
  if (s.n[0] != s.n[1])
    return fail(HFX_EUNSUPPORTED, "grids need n_x == n_y (n_z may differ: slab cells)" + at);
  return HFX_OK;
}

void free_system(SystemPlan& sp) {
  if (sp.vtab) (void)hipFree(sp.vtab);
  for (auto& p : sp.tw)
    if (p) (void)hipFree(p);
  if (sp.d_tiles) (void)hipFree(sp.d_tiles);
  if (sp.d_zero) (void)hipFree(sp.d_zero);
  sp.d_zero = nullptr;
  if (sp.d_active) (void)hipFree(sp.d_active);
  if (sp.d_perm) (void)hipFree(sp.d_perm);
  if (sp.d_keep) (void)hipFree(sp.d_keep);
  sp.d_perm = nullptr;
  sp.d_keep = nullptr;
  if (sp.bstream) (void)hipStreamDestroy(sp.bstream);
  for (hipEvent_t e : {sp.ev_fork, sp.ev_join, sp.ev_acc[0], sp.ev_acc[1]})
    if (e) (void)hipEventDestroy(e);
  sp.vtab = nullptr;
  for (auto& p : sp.tw) p = nullptr;
  sp.d_tiles = nullptr;
  sp.d_active = nullptr;
  sp.bstream = nullptr;
  sp.ev_fork = sp.ev_join = sp.ev_acc[0] = sp.ev_acc[1] = nullptr;
}

// Event bracket around one launch when profiling is on.
struct Bracket {
  hfx_plan plan;
  int pass;
  hipStream_t st;
  hipEvent_t start = nullptr;
  Bracket(hfx_plan p, int ps, hipStream_t s) : plan(p), pass(ps), st(s) {
    if (!plan->prof || plan->capturing || plan->quiet) return;
    start = take_event(plan);
    if (start) (void)hipEventRecord(start, st);
  }
  void done(double bytes, double flops) {
    if (!plan->prof || plan->capturing || plan->quiet || !start) return;
    hipEvent_t stop = take_event(plan);
    if (!stop) return;
    (void)hipEventRecord(stop, st);
    plan->recs.push_back({pass, start, stop, bytes, flops});
    start = nullptr;
  }
  static hipEvent_t take_event(hfx_plan p) {
    hipEvent_t e = nullptr;
    if (!p->pool.empty()) {
      e = p->pool.back();
      p->pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
};

hfx_status check_call(hfx_plan plan, const void* psi, void* ws, size_t ws_bytes) {
  if (!plan) return fail(HFX_EINVAL, "null plan");
  if (!psi) return fail(HFX_EINVAL, "null psi");
  if (!ws && plan->ws_bytes > 0) return fail(HFX_EINVAL, "null workspace");
  if (ws_bytes < plan->ws_bytes)
    return fail(HFX_ENOMEM, "workspace too small: need " + std::to_string(plan->ws_bytes) +
                                " bytes, got " + std::to_string(ws_bytes));
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(HFX_EINVAL, "workspace must be 256-byte aligned");
  return HFX_OK;
}

// Largest share of an orbital's z power beyond the plan's orbital band that
// the input check accepts: such content would change E_x by about this
// relative amount where the band-limited passes skip planes.
constexpr double kBandTolerance = 1e-12;

// Input check (option check=1): every orbital finite, and, for band-limited
// plans, inside the bands the passes rely on: |m| <= k_max / 2 along z (the
// skipped kz planes and the half-length z transform), x (the plane pass's band
// columns) and y (its half-height input).  Host-synchronous (waits for `st`);
// skipped under graph capture.
hfx_status check_inputs(hfx_plan plan, const double* psi, char* ws, hipStream_t st) {
  if (!plan->check || plan->capturing) return HFX_OK;
  for (size_t i = 0; i < plan->sys.size(); ++i) {
    const SystemPlan& sp = plan->sys[i];
    const int nx = sp.sys.n[0], ny = sp.sys.n[1], nz = sp.sys.n[2];
    const int len[3] = {nx, ny, nz};
    const int kmax[3] = {sp.kx_max, sp.ky_max, sp.kz_max};
    const char* name[3] = {"x", "y", "z"};
    double* part = reinterpret_cast<double*>(ws + sp.off_ortho);
    // z first: it also counts the non-finite values
    for (int axis = 2; axis >= 0; --axis) {
      const int m_max = kmax[axis] < len[axis] / 2 ? kmax[axis] / 2 : -1;
      if (axis != 2 && m_max < 0) continue;
      const long long np = check_partials(sp.sys.n_orb, nx, ny, nz, axis);
      if (!launch_check_orbitals(psi + sp.psi_off, sp.sys.n_orb, nx, ny, nz, axis, m_max, part,
                                 st))
        return fail(HFX_EUNSUPPORTED, "input check supports axes of up to 128 points");
      HIP_TRY(hipGetLastError());
      std::vector<double> h((size_t)np * 3);
      HIP_TRY(hipMemcpyAsync(h.data(), part, h.size() * 8, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      const long long per_orb = np / sp.sys.n_orb;
      for (int o = 0; o < sp.sys.n_orb; ++o) {
        double bad = 0.0, tot = 0.0, oob = 0.0;
        for (long long k = 0; k < per_orb; ++k) {
          const double* q = &h[(size_t)(o * per_orb + k) * 3];
          bad += q[0];
          tot += q[1];
          oob += q[2];
        }
        const std::string at = "system " + std::to_string(i) + ", orbital " + std::to_string(o);
        if (bad > 0.0 || !std::isfinite(tot))
          return fail(HFX_EINVAL, "input check: " + at + " holds " +
                                      std::to_string((long long)bad) + " non-finite values");
        // Parseval: sum_k |psi~_k|^2 = len sum psi^2 along every line
        const double frac = tot > 0.0 ? oob / (len[axis] * tot) : 0.0;
        if (m_max >= 0 && !(frac <= kBandTolerance)) {
          char buf[64];
          std::snprintf(buf, sizeof buf, "%.3e", frac);
          return fail(HFX_EINVAL, "input check: " + at + " has " + buf +
                                      " of its power beyond |m_" + name[axis] +
                                      "| <= " + std::to_string(m_max) +
                                      ": the plan's ecut does not hold for these orbitals");
        }
      }
    }
  }
  return HFX_OK;
}

// One system's share of an exchange call: its orbitals (the system's own
// block), K psi destination (its own block; null for the energy only) and
// energy output (nullable).
struct SysCall {
  SystemPlan* sp;
  const double* psi;
  void* kpsi;
  double* ex;
};

// Runs the pair pipeline of the systems of one size class (same kernel
// configuration and band, all screened or none) on stream st.  Each system's
// batches run in order; batch t of every system in the class shares one
// launch per pass (a PassGroup: the systems' workgroup ranges side by side),
// so a class of several systems launches each pass once per batch step
// instead of once per system.  Results equal those of separate launches bit
// for bit (every workgroup does the same work).  acc: accumulate K psi.
hfx_status run_exchange(hfx_plan plan, const std::vector<SysCall>& calls, char* ws,
                        hipStream_t st, bool acc) {
  const Variant* v = calls[0].sp->var;
  const size_t elem = plan->prec == HFX_FP64 ? 8 : 4;
  const int nc = (int)calls.size();
  std::vector<PassArgs> args(nc);
  size_t max_batches = 0;
  // A class of several systems stages, takes the pair means of and zeroes
  // all its members in one launch each (per-system launches on one stream
  // would serialise many small launches); results are those of the
  // per-system launches bit for bit.
  const bool joint = nc > 1;
  if (joint) {
    double orbs = 0.0, mean_flops = 0.0;
    for (const SysCall& c : calls) {
      orbs += (double)c.sp->sys.n_orb * (double)c.sp->nr;
      mean_flops += 2.0 * (double)c.sp->sys.n_orb * c.sp->sys.n_orb * (double)c.sp->nr;
    }
    if (plan->prec == HFX_FP32) {
      std::vector<const double*> in(nc);
      std::vector<float*> out(nc);
      std::vector<size_t> cnt(nc);
      std::vector<int> nn(nc);
      std::vector<long long> nrr(nc);
      std::vector<double> alpha(nc);
      std::vector<double*> part(nc), mu(nc);
      for (int c = 0; c < nc; ++c) {
        SystemPlan& sp = *calls[c].sp;
        in[c] = calls[c].psi;
        out[c] = reinterpret_cast<float*>(ws + sp.off_psi32);
        cnt[c] = (size_t)sp.sys.n_orb * sp.nr;
        nn[c] = sp.sys.n_orb;
        nrr[c] = sp.nr;
        alpha[c] = 1.0 / (double)sp.nr;
        part[c] = reinterpret_cast<double*>(ws + sp.off_gemm);
        mu[c] = reinterpret_cast<double*>(ws + sp.off_mean);
      }
      {
        Bracket br(plan, HFX_PASS_STAGE, st);
        launch_cast_group(in.data(), out.data(), cnt.data(), nc, st);
        br.done(orbs * 12.0, 0.0);
      }
      Bracket br(plan, HFX_PASS_CONTRACT, st);
      launch_gram_self_group(in.data(), nn.data(), nrr.data(), alpha.data(), part.data(),
                             mu.data(), nc, st);
      for (int c = 0; c < nc; ++c)
        if (calls[c].sp->d_keep)
          launch_mask(mu[c], calls[c].sp->d_keep,
                      (size_t)calls[c].sp->sys.n_orb * calls[c].sp->sys.n_orb, st);
      br.done(orbs * 8.0, mean_flops);
    }
    if (acc) {
      std::vector<void*> dst(nc);
      std::vector<size_t> bytes(nc);
      for (int c = 0; c < nc; ++c) {
        dst[c] = calls[c].kpsi;
        bytes[c] = (size_t)calls[c].sp->sys.n_orb * calls[c].sp->nr * elem;
      }
      Bracket br(plan, HFX_PASS_ZERO, st);
      launch_zero_group(dst.data(), bytes.data(), nc, st);
      br.done(orbs * elem, 0.0);
    }
  }
  for (int c = 0; c < nc; ++c) {
    SystemPlan& sp = *calls[c].sp;
    const double* psi = calls[c].psi;
    const void* psi_w = psi;
    const double orb_pts = (double)sp.sys.n_orb * (double)sp.nr;
    if (joint) {
      psi_w = plan->prec == HFX_FP32 ? static_cast<const void*>(ws + sp.off_psi32) : psi;
    } else if (plan->prec == HFX_FP32) {
      float* p32 = reinterpret_cast<float*>(ws + sp.off_psi32);
      Bracket br(plan, HFX_PASS_STAGE, st);
      launch_cast_f64_f32(psi, p32, (size_t)sp.sys.n_orb * sp.nr, st);
      br.done(orb_pts * 12.0, 0.0);
      psi_w = p32;
    }
    // float32 plans: exact pair-density means mu_ab = (1/N_r) sum_r psi_a psi_b
    // (float64 MFMA).  Transforming rho_ab - mu_ab keeps the large G = 0
    // coefficient out of the float32 FFTs; v(0) mu_ab is added back to the
    // potentials and v(0) Omega mu_ab^2 to the energy in float64.
    const double* mean = nullptr;
    if (joint) {
      if (plan->prec == HFX_FP32) mean = reinterpret_cast<double*>(ws + sp.off_mean);
    } else if (plan->prec == HFX_FP32) {
      double* mu = reinterpret_cast<double*>(ws + sp.off_mean);
      double* part = reinterpret_cast<double*>(ws + sp.off_gemm);
      Bracket br(plan, HFX_PASS_CONTRACT, st);
      launch_xtx_f64(psi, psi, sp.sys.n_orb, sp.nr, 1.0 / (double)sp.nr, part, mu, st);
      // screened pairs contribute no G = 0 energy either
      if (sp.d_keep) launch_mask(mu, sp.d_keep, (size_t)sp.sys.n_orb * sp.sys.n_orb, st);
      br.done(orb_pts * 8.0, 2.0 * (double)sp.sys.n_orb * orb_pts);
      mean = mu;
    }
    if (acc && !joint) {
      Bracket br(plan, HFX_PASS_ZERO, st);
      launch_zero(calls[c].kpsi, (size_t)sp.sys.n_orb * sp.nr * elem, st);
      br.done(orb_pts * elem, 0.0);
    }
    PassArgs& a = args[c];
    a = PassArgs{};
    a.psi = psi_w;
    a.kpsi = calls[c].kpsi;
    a.vtab = sp.vtab;
    a.tw_zf = sp.tw[0];
    a.tw_zi = sp.tw[1];
    a.tw_xf = sp.tw[2];
    a.tw_xi = sp.tw[3];
    a.tw_yf = sp.tw[4];
    a.tw_yi = sp.tw[5];
    a.tw_zh = sp.tw[6];
    a.partials = reinterpret_cast<double*>(ws + sp.off_partials);
    a.mean = mean;
    a.v0 = sp.v0;
    a.perm = sp.d_perm;
    a.n_orb = sp.sys.n_orb;
    a.kz_max = sp.kz_max;
    a.kx_max = sp.kx_max;
    a.ky_max = sp.ky_max;
    a.zero = sp.d_zero;
    max_batches = std::max(max_batches, sp.batches.size());
  }
  const int br = bricks_per_tile(v);
  const int n = v->n, nz = v->nz;
  const int nxb = (n + v->brick - 1) / v->brick;
  const double ce = 2.0 * elem;  // complex element bytes
  // Two batch streams (single-system classes only): batch k runs on stream
  // k % 2 with grid buffer k % 2.  Its inv_acc waits for batch k-1's, so K
  // psi receives its updates in the serial order (identical results) while
  // the transforms of one batch overlap the other batch's passes.
  // Consecutive batches of one tile round touch disjoint orbitals anyway;
  // across rounds the wait is needed.  Graph capture keeps the batches on
  // the one stream (the two-stream form is not captured): a captured graph
  // equals that of a streams=1 plan.
  SystemPlan& sp0 = *calls[0].sp;
  const bool two = nc == 1 && sp0.nstreams == 2 && sp0.batches.size() > 1 && !plan->capturing;
  if (two) {
    HIP_TRY(hipEventRecord(sp0.ev_fork, st));
    HIP_TRY(hipStreamWaitEvent(sp0.bstream, sp0.ev_fork, 0));
  }
  for (size_t k = 0; k < max_batches; ++k) {
    const int q = two ? (int)(k & 1) : 0;
    const hipStream_t bs = q ? sp0.bstream : st;
    // the systems with a batch k, their workgroups per pass, and the
    // algorithmic bytes and flops of each pass over them
    PassGroup g{};
    std::vector<int> who;
    double by_fwd = 0, fl_fwd = 0, by_pl = 0, fl_pl = 0, by_row = 0, fl_row = 0, by_col = 0,
           fl_col = 0, by_inv = 0, fl_inv = 0;
    std::vector<int> nb_fwd, nb_pl, nb_row, nb_col, nb_inv;
    // half-height plane input: a decision for the whole launch, as the
    // kernels' launchers take it
    bool hy = v->hy, xd = v->xd;
    for (int c = 0; c < nc; ++c)
      if (k < calls[c].sp->batches.size()) {
        hy = hy && half_y(v, calls[c].sp->kx_max, calls[c].sp->ky_max);
        xd = xd && half_x(v, calls[c].sp->kx_max, calls[c].sp->ky_max);
      }
    const double yf = hy ? 0.5 : 1.0;  // share of the rows pass 1 runs on
    const double xf = xd ? 0.5 : 1.0;  // share of the columns it stores
    const int nxbh = (n / 2 + v->brick - 1) / v->brick;  // bricks per half-width row
    for (int c = 0; c < nc; ++c) {
      SystemPlan& sp = *calls[c].sp;
      if (k >= sp.batches.size()) continue;
      const Batch& b = sp.batches[k];
      PassArgs a = args[c];
      a.grids = ws + sp.off_grids + (size_t)q * sp.grid_bytes;
      a.tiles = sp.d_tiles + b.tile_off;
      a.active = sp.d_active + b.active_off;
      a.n_tiles = b.n_tiles;
      a.n_active = b.n_active;
      a.part_base = b.part_base;
      g.a[(int)who.size()] = a;
      who.push_back(c);
      const double nr = (double)sp.nr;
      // share of the grid on kept kz planes (pair-grid traffic of the passes)
      const double kzf = (double)kz_planes(nz, sp.kz_max) / nz;
      // FFT flops per complex grid and axis pass: 5 N_r log2(N) (radix-2 count)
      const double fft_axis = 5.0 * nr * std::log2((double)n);  // x or y
      const double fft_z = 5.0 * nr * std::log2((double)nz);
      double orbs = 0.0;  // orbital rows a batch reads (each tile's blocks once)
      for (int t = 0; t < b.n_tiles; ++t) {
        const TileDesc& td = sp.tiles[b.tile_off + t];
        if (sp.d_keep) {
          // screened: only rows and columns with an evaluated pair are touched
          // (in a diagonal tile, column b is row joff + b)
          unsigned long long rows = 0, cols = 0;
          for (int r = 0; r < td.nI; ++r)
            for (int cc = 0; cc < td.nJ; ++cc)
              if (keep_bit(td, r, cc)) {
                rows |= 1ull << r;
                cols |= 1ull << (td.diag ? td.joff + cc : cc);
              }
          orbs += td.diag ? __builtin_popcountll(rows | cols)
                          : __builtin_popcountll(rows) + __builtin_popcountll(cols);
        } else {
          orbs += td.diag ? td.nI : td.nI + td.nJ;  // J lies inside I's rows
        }
      }
      const double grids = (double)b.n_active;
      const int kp = kz_planes(nz, sp.kz_max);
      nb_fwd.push_back(b.n_tiles * (xd ? (n / 2) * nxbh : hy ? (n / 2) * nxb : br));
      // a half-length forward z transform reads the orbitals on even z only,
      // half-height input on even y only (and stores half the rows);
      // half-width input stores half the columns (its orbital reads, every
      // other point of a row, still move whole rows)
      by_fwd += orbs * nr * elem * (half_z(v, sp.kz_max) ? 0.5 : 1.0) * yf +
                grids * nr * ce * kzf * yf * xf;
      fl_fwd += grids * fft_z * yf * xf;
      nb_pl.push_back(b.n_active * kp);
      by_pl += grids * nr * ce * (1.0 + yf * xf) * kzf;
      fl_pl += grids * fft_axis * 4.0 * kzf;
      nb_row.push_back(b.n_active * ((kp * n + v->rows_per_wg - 1) / std::max(v->rows_per_wg, 1)));
      by_row += grids * nr * ce * 2.0 * kzf;
      fl_row += grids * fft_axis * kzf;
      nb_col.push_back(b.n_active * kp * nxb);
      by_col += grids * nr * ce * 2.0 * kzf;
      fl_col += grids * fft_axis * 2.0 * kzf;
      nb_inv.push_back(b.n_tiles * br);
      by_inv += grids * nr * ce * kzf + orbs * nr * elem * (acc ? 3.0 : 1.0);
      fl_inv += grids * fft_z;
    }
    g.count = (int)who.size();
    auto launch = [&](launch_fn fn, const std::vector<int>& nbs, int pass, double bytes,
                      double flops) {
      int total = 0;
      for (int i = 0; i < g.count; ++i) {
        g.start[i] = total;
        total += nbs[i];
      }
      g.start[g.count] = total;
      Bracket bk(plan, pass, bs);
      fn(g, total, bs);
      bk.done(bytes, flops);
    };
    launch(v->pair_fwd, nb_fwd, HFX_PASS_PAIR_FWD, by_fwd, fl_fwd);
    if (v->plane_mode == 0) {
      launch(v->plane, nb_pl, HFX_PASS_PLANE, by_pl, fl_pl);
    } else {
      // rows and planes of the kept kz planes only
      launch(v->rows_fwd, nb_row, HFX_PASS_ROWS_FWD, by_row, fl_row);
      launch(v->cols_conv, nb_col, HFX_PASS_COLS_CONV, by_col, fl_col);
      launch(v->rows_inv, nb_row, HFX_PASS_ROWS_INV, by_row, fl_row);
    }
    if (two && k > 0) HIP_TRY(hipStreamWaitEvent(bs, sp0.ev_acc[q ^ 1], 0));
    if (acc)
      launch(v->inv_acc, nb_inv, HFX_PASS_INV_ACC, by_inv, fl_inv);
    else
      launch(v->inv_energy, nb_inv, HFX_PASS_INV_ENERGY, by_inv, fl_inv);
    if (two) HIP_TRY(hipEventRecord(sp0.ev_acc[q], bs));
  }
  if (two) {
    HIP_TRY(hipEventRecord(sp0.ev_join, sp0.bstream));
    HIP_TRY(hipStreamWaitEvent(st, sp0.ev_join, 0));
  }
  for (int c = 0; c < nc; ++c) {
    if (!calls[c].ex) continue;
    SystemPlan& sp = *calls[c].sp;
    Bracket bk(plan, HFX_PASS_ENERGY_REDUCE, st);
    const double om = sp.dv * (double)sp.nr;
    // the G = 0 energy of the means is not pair work: added by group 0 only
    const bool dc = sp.shard == 0;
    launch_energy_reduce(args[c].partials, sp.n_partials, -0.5 * sp.dv,
                         dc ? args[c].mean : nullptr, sp.sys.n_orb,
                         dc ? -0.5 * om * sp.v0 : 0.0, calls[c].ex, st);
    bk.done((double)sp.n_partials * 8.0, 0.0);
  }
  HIP_TRY(hipGetLastError());
  return HFX_OK;
}

// Largest pair_fwd launch of a system's schedule, in workgroups.
long long largest_launch(const SystemPlan& sp) {
  long long m = 0;
  for (const Batch& b : sp.batches) m = std::max<long long>(m, b.n_tiles);
  return m * bricks_per_tile(sp.var);
}

// Systems whose pass launches stay below this many workgroups (two per
// compute unit) join size classes by default: their own launches leave the
// device partly idle and the per-launch costs dominate.  Larger systems do
// better as separate launch sequences on forked streams, where different
// passes of different systems overlap (measured on one MI355X: 16 systems
// of 8-23 orbitals on 24^3, 0.70 ms shared against 1.26 ms forked; 8 of
// 32 orbitals on 96^3, 15.7 against 15.2 ms).
constexpr long long kGroupBelowWorkgroups = 512;

// The size classes of a plan's systems for the exchange calls: systems with
// the same kernel configuration, band and screening state share launches
// (at most kMaxGroup per class).  A system with two batch streams, one of a
// plan created with group=0, or (by default) one whose own launches are
// large, is a class of its own; group=1 groups every system it can.
// Classes keep the plan order of their first system.
std::vector<std::vector<int>> size_classes(hfx_plan plan) {
  std::vector<std::vector<int>> out;
  for (int i = 0; i < (int)plan->sys.size(); ++i) {
    const SystemPlan& sp = plan->sys[i];
    bool placed = false;
    const bool groupable =
        plan->group == 1 || (plan->group < 0 && largest_launch(sp) < kGroupBelowWorkgroups);
    if (groupable && sp.nstreams == 1 && !sp.var->persistent)
      for (auto& c : out) {
        const SystemPlan& f = plan->sys[c[0]];
        const bool fg =
            plan->group == 1 || (plan->group < 0 && largest_launch(f) < kGroupBelowWorkgroups);
        if ((int)c.size() < kMaxGroup && fg && f.var == sp.var && f.kz_max == sp.kz_max &&
            (f.d_keep != nullptr) == (sp.d_keep != nullptr) && f.nstreams == 1 &&
            !f.var->persistent) {
          c.push_back(i);
          placed = true;
          break;
        }
      }
    if (!placed) out.push_back({i});
  }
  return out;
}

// ---------------------------------------------------------------------------
// Per-system launch sequences of each entry point.

// Exchange calls of one size class (cls: system indices).  psi, kpsi, grad
// and ex are the call's concatenated buffers.
hfx_status enq_energy(hfx_plan plan, const std::vector<int>& cls, const double* psi, double* ex,
                      char* ws, hipStream_t st) {
  std::vector<SysCall> calls;
  for (int i : cls) {
    SystemPlan& sp = plan->sys[i];
    calls.push_back({&sp, psi + sp.psi_off, nullptr, ex + i});
  }
  return run_exchange(plan, calls, ws, st, false);
}

hfx_status enq_apply(hfx_plan plan, const std::vector<int>& cls, const double* psi, void* kpsi,
                     double* ex, char* ws, hipStream_t st) {
  const size_t elem = plan->prec == HFX_FP64 ? 8 : 4;
  std::vector<SysCall> calls;
  for (int i : cls) {
    SystemPlan& sp = plan->sys[i];
    calls.push_back({&sp, psi + sp.psi_off, static_cast<char*>(kpsi) + (size_t)sp.psi_off * elem,
                     ex ? ex + i : nullptr});
  }
  return run_exchange(plan, calls, ws, st, true);
}

hfx_status enq_gradient(hfx_plan plan, const std::vector<int>& cls, const double* psi,
                        const double* gscale, double* grad, char* ws, hipStream_t st) {
  std::vector<SysCall> calls;
  for (int i : cls) {
    SystemPlan& sp = plan->sys[i];
    double* g = grad + sp.psi_off;
    void* kp = plan->prec == HFX_FP64 ? static_cast<void*>(g) : static_cast<void*>(ws + sp.off_kpsi);
    calls.push_back({&sp, psi + sp.psi_off, kp, nullptr});
  }
  hfx_status s = run_exchange(plan, calls, ws, st, true);
  if (s != HFX_OK) return s;
  for (size_t c = 0; c < cls.size(); ++c) {
    SystemPlan& sp = *calls[c].sp;
    Bracket bk(plan, HFX_PASS_SCALE, st);
    launch_scale_to_f64(calls[c].kpsi, plan->prec == HFX_FP64, grad + sp.psi_off,
                        (size_t)sp.sys.n_orb * sp.nr, 2.0 * sp.dv,
                        gscale ? gscale + cls[c] : nullptr, st);
    bk.done((double)sp.sys.n_orb * sp.nr * (plan->prec == HFX_FP64 ? 16.0 : 12.0), 0.0);
  }
  HIP_TRY(hipGetLastError());
  return HFX_OK;
}

// M of one system from its own K psi block kp (not a concatenated buffer).
hfx_status enq_matrix_sys(hfx_plan plan, SystemPlan& sp, const double* psi, const void* kp_sys,
                          double* m, char* ws, hipStream_t st) {
  const size_t elem = plan->prec == HFX_FP64 ? 8 : 4;
  double* part = reinterpret_cast<double*>(ws + sp.off_gemm);
  const char* kp = static_cast<const char*>(kp_sys);
  const double nn = (double)sp.sys.n_orb, npts = (double)sp.nr;
  Bracket bk(plan, HFX_PASS_CONTRACT, st);
  if (plan->prec == HFX_FP32)
    launch_xtx_split(psi + sp.psi_off, reinterpret_cast<const float*>(kp), sp.sys.n_orb, sp.nr,
                     sp.dv, part, m + sp.m_off, st);
  else
    launch_xtx_f64(psi + sp.psi_off, reinterpret_cast<const double*>(kp), sp.sys.n_orb, sp.nr,
                   sp.dv, part, m + sp.m_off, st);
  // split precision: two float32 products per term
  bk.done(nn * npts * (8.0 + elem), 2.0 * nn * nn * npts * (plan->prec == HFX_FP32 ? 2.0 : 1.0));
  HIP_TRY(hipGetLastError());
  return HFX_OK;
}

hfx_status enq_matrix(hfx_plan plan, SystemPlan& sp, const double* psi, const void* kpsi,
                      double* m, char* ws, hipStream_t st) {
  const size_t elem = plan->prec == HFX_FP64 ? 8 : 4;
  return enq_matrix_sys(plan, sp, psi, static_cast<const char*>(kpsi) + (size_t)sp.psi_off * elem,
                        m, ws, st);
}

// K psi into the workspace, then M from it (and E_x when ex is given).
hfx_status enq_matrix_full(hfx_plan plan, const std::vector<int>& cls, const double* psi,
                           double* m, double* ex, char* ws, hipStream_t st) {
  std::vector<SysCall> calls;
  for (int i : cls) {
    SystemPlan& sp = plan->sys[i];
    calls.push_back({&sp, psi + sp.psi_off, ws + sp.off_kpsi, ex ? ex + i : nullptr});
  }
  hfx_status r = run_exchange(plan, calls, ws, st, true);
  for (size_t c = 0; c < calls.size() && r == HFX_OK; ++c)
    r = enq_matrix_sys(plan, *calls[c].sp, psi, calls[c].kpsi, m, ws, st);
  return r;
}

// ACE projectors: L = chol(-M), X = L^(-1), P = X W (Eq. (vx_ace)).
hfx_status enq_ace_build(hfx_plan plan, SystemPlan& sp, const void* kpsi, const double* m,
                         double* p, char* ws, hipStream_t st) {
  const int n = sp.sys.n_orb;
  const size_t elem = plan->prec == HFX_FP64 ? 8 : 4;
  double* work = reinterpret_cast<double*>(ws + sp.off_ortho);
  double* low = work;                      // n x n
  double* inv = work + (size_t)n * n;      // n x n
  double* tmp = reinterpret_cast<double*>(ws + align_up(sp.off_ortho + (size_t)6 * n * n * 8 + 64));
  const char* kp = static_cast<const char*>(kpsi) + (size_t)sp.psi_off * elem;
  double* pp = p + sp.psi_off;
  const double nn = n, npts = (double)sp.nr;
  Bracket bk(plan, HFX_PASS_ACE_BUILD, st);
  launch_chol(m + sp.m_off, n, -1.0, low, st);
  launch_trinv(low, n, inv, st);
  if (plan->prec == HFX_FP64) {
    // P = X W straight from the float64 K psi
    launch_apply_left(inv, reinterpret_cast<const double*>(kp), pp, n, sp.nr, tmp, st);
    bk.done(nn * npts * 16.0, 2.0 * nn * nn * npts);
  } else if (launch_apply_left_f32(inv, reinterpret_cast<const float*>(kp), pp, n, sp.nr, st)) {
    // float32 K psi widened while staged
    bk.done(nn * npts * (elem + 8.0), 2.0 * nn * nn * npts);
  } else {
    // larger sets: widen into P, then P <- X P in place
    launch_scale_to_f64(kp, 0, pp, (size_t)n * sp.nr, 1.0, nullptr, st);
    launch_apply_left(inv, pp, pp, n, sp.nr, tmp, st);
    bk.done(nn * npts * (elem + 8.0 + 16.0), 2.0 * nn * nn * npts);
  }
  HIP_TRY(hipGetLastError());
  return HFX_OK;
}

// out = V^ACE phi = -sum_k P_k <P_k|phi>: G = -dV phi P^T, out = G P.
hfx_status enq_ace_apply(hfx_plan plan, SystemPlan& sp, const double* p, const double* phi,
                         double* out, char* ws, hipStream_t st) {
  const int n = sp.sys.n_orb;
  double* part = reinterpret_cast<double*>(ws + sp.off_gemm);
  double* g = reinterpret_cast<double*>(ws + sp.off_ortho) + (size_t)2 * n * n;
  double* tmp = reinterpret_cast<double*>(ws + align_up(sp.off_ortho + (size_t)6 * n * n * 8 + 64));
  const double nn = n, npts = (double)sp.nr;
  Bracket bk(plan, HFX_PASS_ACE_APPLY, st);
  launch_xtx_f64(phi + sp.psi_off, p + sp.psi_off, n, sp.nr, -sp.dv, part, g, st);
  launch_apply_left(g, p + sp.psi_off, out + sp.psi_off, n, sp.nr, tmp, st);
  bk.done(nn * npts * 8.0 * 4.0, 4.0 * nn * nn * npts);
  HIP_TRY(hipGetLastError());
  return HFX_OK;
}

hfx_status enq_ortho(hfx_plan plan, SystemPlan& sp, double* psi, int method, char* ws,
                     hipStream_t st) {
  const int n = sp.sys.n_orb;
  double* part = reinterpret_cast<double*>(ws + sp.off_gemm);
  double* work = reinterpret_cast<double*>(ws + sp.off_ortho);
  double* smat = work;                     // n x n overlap, replaced by S^(-1/2)
  double* ns_work = work + (size_t)n * n;  // 5 n^2 doubles + flags
  double* tmp = reinterpret_cast<double*>(ws + align_up(sp.off_ortho + (size_t)6 * n * n * 8 + 64));
  double* p = psi + sp.psi_off;
  const double nn = n, npts = (double)sp.nr;
  {
    Bracket bk(plan, HFX_PASS_CONTRACT, st);
    launch_xtx_f64(p, p, n, sp.nr, sp.dv, part, smat, st);
    bk.done(nn * npts * 8.0, 2.0 * nn * nn * npts);
  }
  Bracket bk(plan, HFX_PASS_ORTHO, st);
  if (method == HFX_ORTHO_CHOLESKY) {
    // S = L L^T, Psi <- L^(-1) Psi
    double* low = work + (size_t)n * n;
    double* inv = work + (size_t)2 * n * n;
    launch_chol(smat, n, 1.0, low, st);
    launch_trinv(low, n, inv, st);
    launch_apply_left(inv, p, p, n, sp.nr, tmp, st);
  } else {
    HIP_TRY(launch_inverse_sqrt(smat, n, ns_work, 40, st));
    launch_apply_left(smat, p, p, n, sp.nr, tmp, st);
  }
  bk.done(nn * npts * 16.0, 2.0 * nn * nn * npts);
  HIP_TRY(hipGetLastError());
  return HFX_OK;
}

// SCDM-localised orthonormal orbitals: pivots by column-pivoted QR of
// Psi^T, density-matrix columns B Psi with b[k][i] = psi_i(c_k), then Loewdin.
// Scratch: the pair-grid buffer (w and the argmax candidates, unused outside
// the exchange calls) and the orthonormalisation region (q rows and B).
hfx_status enq_scdm(hfx_plan plan, SystemPlan& sp, const double* psi, double* phi, int* pivots,
                    char* ws, hipStream_t st) {
  const int n = sp.sys.n_orb;
  char* scratch = ws + sp.off_grids;
  double* work = reinterpret_cast<double*>(ws + sp.off_ortho);
  double* qm = work;
  double* b = work + (size_t)n * n;
  double* tmp = reinterpret_cast<double*>(ws + align_up(sp.off_ortho + (size_t)6 * n * n * 8 + 64));
  int* piv = pivots ? pivots + sp.orb_off
                    : reinterpret_cast<int*>(scratch + align_up(scdm_scratch_bytes(sp.nr)));
  const double* ps = psi + sp.psi_off;
  double* ph = phi + sp.psi_off;
  const double nn = n, npts = (double)sp.nr;
  {
    Bracket bk(plan, HFX_PASS_SCDM, st);
    launch_scdm_pivots(ps, n, sp.nr, scratch, qm, piv, st);
    launch_scdm_gather(ps, n, sp.nr, piv, b, st);
    launch_apply_left(b, ps, ph, n, sp.nr, tmp, st);
    // every pivot step reads Psi once; the columns B Psi read and write it
    bk.done(nn * npts * 8.0 * (nn + 2.0), 2.0 * nn * npts * (nn + 1.0) + 2.0 * nn * nn * npts);
  }
  HIP_TRY(hipGetLastError());
  return enq_ortho(plan, sp, phi, HFX_ORTHO_LOWDIN, ws, st);
}

// Runs fn(system, stream) for every system.  One system: on the caller's
// stream.  Several: forked onto the plan's side streams after an event on the
// caller's stream and joined back with one event per system, so independent
// systems overlap while the call keeps stream semantics.
template <class F>
hfx_status dispatch(hfx_plan plan, hipStream_t user, F&& fn) {
  if (plan->sys.size() == 1) return fn(0, user);
  HIP_TRY(hipEventRecord(plan->fork, user));
  for (size_t i = 0; i < plan->sys.size(); ++i) {
    HIP_TRY(hipStreamWaitEvent(plan->side[i], plan->fork, 0));
    hfx_status s = fn(i, plan->side[i]);
    if (s != HFX_OK) return s;
    HIP_TRY(hipEventRecord(plan->join[i], plan->side[i]));
    HIP_TRY(hipStreamWaitEvent(user, plan->join[i], 0));
  }
  return HFX_OK;
}

// Runs fn(class, stream) for every size class of the plan's systems (see
// size_classes): one class on the caller's stream, several forked onto the
// side streams of their first systems and joined back like dispatch().
template <class F>
hfx_status dispatch_classes(hfx_plan plan, hipStream_t user, F&& fn) {
  const std::vector<std::vector<int>> classes = size_classes(plan);
  if (classes.size() == 1) return fn(classes[0], user);
  HIP_TRY(hipEventRecord(plan->fork, user));
  for (const auto& cls : classes) {
    const int i = cls[0];
    HIP_TRY(hipStreamWaitEvent(plan->side[i], plan->fork, 0));
    hfx_status s = fn(cls, plan->side[i]);
    if (s != HFX_OK) return s;
    HIP_TRY(hipEventRecord(plan->join[i], plan->side[i]));
    HIP_TRY(hipStreamWaitEvent(user, plan->join[i], 0));
  }
  return HFX_OK;
}

}  // namespace

extern "C" {

const char* hfx_status_string(hfx_status s) {
  switch (s) {
    case HFX_OK: return "HFX_OK";
    case HFX_EINVAL: return "HFX_EINVAL: invalid argument";
    case HFX_EUNSUPPORTED: return "HFX_EUNSUPPORTED: unsupported configuration";
    case HFX_ENOMEM: return "HFX_ENOMEM: insufficient memory";
    case HFX_EDEVICE: return "HFX_EDEVICE: HIP runtime error";
  }
  return "unknown hfx_status";
}

const char* hfx_last_error(void) { return g_last_error.c_str(); }

const char* hfx_variants(int n, int precision) {
  static thread_local std::string out;
  out.clear();
  int count = 0;
  const Variant* v = precision == HFX_FP64 ? variants_f64(&count) : variants_f32(&count);
  for (int i = 0; i < count; ++i)
    if (v[i].n == n && v[i].nz == n) {  // cubic grids
      if (!out.empty()) out += ";";
      out += v[i].name;
    }
  return out.c_str();
}

hfx_status hfx_plan_create(hfx_plan* out, const hfx_system* sys, int n_sys, int precision,
                           const char* options) {
  g_last_error.clear();
  if (!out) return fail(HFX_EINVAL, "null output plan pointer");
  *out = nullptr;
  if (!sys) return fail(HFX_EINVAL, "null system array");
  if (n_sys < 1) return fail(HFX_EINVAL, "n_sys must be >= 1");
  if (precision != HFX_FP32 && precision != HFX_FP64)
    return fail(HFX_EINVAL, "precision must be HFX_FP32 or HFX_FP64");
  for (int i = 0; i < n_sys; ++i) {
    hfx_status s = validate_system(sys[i], i);
    if (s != HFX_OK) return s;
    if (!find_variant(sys[i].n[0], sys[i].n[2], precision))
      return fail(HFX_EUNSUPPORTED, "grid " + std::to_string(sys[i].n[0]) + "^2 x " +
                                        std::to_string(sys[i].n[2]) +
                                        " is not supported (system " + std::to_string(i) +
                                        ")");
  }
  {
    std::string bad;
    if (!options_known(options, &bad))
      return fail(HFX_EINVAL, "unknown plan option '" + bad + "'");
  }
  long long ws_cap = 0, batch_streams = 1;
  if (!parse_option(options, "maxws", 0, &ws_cap))
    return fail(HFX_EINVAL, "maxws= takes a non-negative integer (bytes)");
  if (!parse_option(options, "streams", 1, &batch_streams))
    return fail(HFX_EINVAL, "streams= must be 1 or 2");
  long long group_opt = -1;
  if (has_option(options, "group") &&
      (!parse_option(options, "group", -1, &group_opt) || group_opt > 1))
    return fail(HFX_EINVAL, "group= takes 0 or 1");
  long long check_opt = 0;
  if (!parse_option(options, "check", 0, &check_opt) || check_opt > 1)
    return fail(HFX_EINVAL, "check= takes 0 or 1");
  if (!has_option(options, "check"))
    if (const char* env = std::getenv("HFX_CHECK_INPUTS"))
      check_opt = (*env && std::strcmp(env, "0") != 0) ? 1 : 0;
  int shard = 0, shards = 1;
  {
    const std::string sv = parse_option_str(options, "shard");
    if (!sv.empty()) {
      const size_t slash = sv.find('/');
      if (slash == std::string::npos)
        return fail(HFX_EINVAL, "shard= takes <group>/<groups>");
      shard = std::atoi(sv.substr(0, slash).c_str());
      shards = std::atoi(sv.substr(slash + 1).c_str());
      if (shards < 1 || shard < 0 || shard >= shards)
        return fail(HFX_EINVAL, "shard=<g>/<R> needs 0 <= g < R");
    }
  }
  double mix = 1.0;
  {
    const std::string mv = parse_option_str(options, "mix");
    if (mv.empty() && has_option(options, "mix"))
      return fail(HFX_EINVAL, "mix=<a> needs 0 < a <= 1");
    if (!mv.empty()) {
      char* end = nullptr;
      mix = std::strtod(mv.c_str(), &end);
      if (end == mv.c_str() || *end != '\0' || !(mix > 0.0 && mix <= 1.0))
        return fail(HFX_EINVAL, "mix=<a> needs 0 < a <= 1");
    }
  }
  double ecut = 0.0;
  {
    const std::string ev = parse_option_str(options, "ecut");
    if (ev.empty() && has_option(options, "ecut"))
      return fail(HFX_EINVAL, "ecut=<Ha> needs a positive cutoff");
    if (!ev.empty()) {
      char* end = nullptr;
      ecut = std::strtod(ev.c_str(), &end);
      if (end == ev.c_str() || *end != '\0' || !(ecut > 0.0 && ecut < 1e6))
        return fail(HFX_EINVAL, "ecut=<Ha> needs a positive cutoff");
    }
  }
  // Per-system kernel configuration: variant=, tiles= and rows= take one
  // value for every system or a ','-separated list with one per system;
  // systems that name none take the tune cache's choice, else the defaults.
  std::vector<std::string> vnames(n_sys);
  std::vector<long long> tiles_v(n_sys, 0), rows_v(n_sys, 0);
  std::vector<char> tuned(n_sys, 0);
  {
    const std::string vv = parse_option_str(options, "variant");
    const std::string tv = parse_option_str(options, "tiles");
    const std::string rv = parse_option_str(options, "rows");
    if (tv.empty() && has_option(options, "tiles"))
      return fail(HFX_EINVAL, "tiles= takes a non-negative integer");
    if (rv.empty() && has_option(options, "rows"))
      return fail(HFX_EINVAL, "rows= takes 8, 16, 24 or 32");
    std::string tc = parse_option_str(options, "tune_cache");
    if (tc.empty() && has_option(options, "tune_cache"))
      return fail(HFX_EINVAL, "tune_cache= needs a file path");
    if (tc.empty())
      if (const char* env = std::getenv("HFX_AUTOTUNE_CACHE")) tc = env;
    double ecut_k = 0.0;
    {
      const std::string ev = parse_option_str(options, "ecut");
      if (!ev.empty()) ecut_k = std::strtod(ev.c_str(), nullptr);
    }
    for (int i = 0; i < n_sys; ++i) {
      std::string x;
      if (!per_system_value(vv, i, n_sys, &x))
        return fail(HFX_EINVAL, "variant= list needs one name per system");
      vnames[i] = x;
      if (!per_system_value(tv, i, n_sys, &x) || (!x.empty() && !parse_count(x, &tiles_v[i])))
        return fail(HFX_EINVAL, "tiles= takes a non-negative integer (or one per system)");
      if (!per_system_value(rv, i, n_sys, &x) || (!x.empty() && !parse_count(x, &rows_v[i])) ||
          (rows_v[i] != 0 && (rows_v[i] % 8 != 0 || rows_v[i] > kMaxRows)))
        return fail(HFX_EINVAL, "rows= takes 8, 16, 24 or 32 (or one per system)");
      if (!tc.empty()) {
        std::string topt;
        int dev = 0;
        (void)hipGetDevice(&dev);
        const std::string key =
            tune_key(sys[i], precision, kz_max_for(ecut_k, sys[i].L[2]), device_arch(dev));
        if (tune_lookup(tc, key, &topt)) {
          // explicit options win over the cache
          const std::string cv = parse_option_str(topt.c_str(), "variant");
          const std::string ct = parse_option_str(topt.c_str(), "tiles");
          const std::string cr = parse_option_str(topt.c_str(), "rows");
          long long t = 0, r = 0;
          if (vnames[i].empty() && !cv.empty() &&
              find_variant(sys[i].n[0], sys[i].n[2], precision, cv))
            vnames[i] = cv;
          if (tv.empty() && parse_count(ct, &t)) tiles_v[i] = t;
          if (rv.empty() && parse_count(cr, &r) && r % 8 == 0 && r <= kMaxRows) rows_v[i] = r;
          tuned[i] = 1;
        }
      }
      if (!vnames[i].empty() && !find_variant(sys[i].n[0], sys[i].n[2], precision, vnames[i]))
        return fail(HFX_EINVAL, "unknown variant '" + vnames[i] + "' for the grid of system " +
                                    std::to_string(i));
    }
  }
  if (batch_streams != 1 && batch_streams != 2)
    return fail(HFX_EINVAL, "streams= must be 1 or 2");
  if (const char* env = std::getenv("HFX_MAX_WORKSPACE_BYTES")) {
    const long long e = std::atoll(env);
    if (e > 0) ws_cap = ws_cap > 0 ? std::min(ws_cap, e) : e;
  }

  hfx_plan p = new hfx_plan_t();
  p->prec = precision;
  p->check = check_opt == 1;
  p->group = (int)group_opt;
  p->sys.resize(n_sys);
  size_t off = 0;
  long long psi_off = 0, m_off = 0, orb_off = 0;
  const size_t elem = precision == HFX_FP64 ? 8 : 4;
  for (int i = 0; i < n_sys; ++i) {
    SystemPlan& sp = p->sys[i];
    sp.sys = sys[i];
    sp.var = find_variant(sys[i].n[0], sys[i].n[2], precision, vnames[i]);
    sp.tuned = tuned[i] != 0;
    sp.n = sys[i].n[0];
    sp.nr = (long long)sp.n * sp.n * sys[i].n[2];
    sp.dv = sys[i].L[0] * sys[i].L[1] * sys[i].L[2] / (double)sp.nr;
    sp.shard = shard;
    sp.shards = shards;
    sp.tiles_cap = tiles_v[i];
    {
      // rows per tile pair: a multiple of the tile, at most what the variant
      // allows (rows= is clamped per system)
      const int t = sp.var->tile;
      int r = rows_v[i] > 0 ? (int)rows_v[i] : default_rows(sp.sys.n_orb);
      r = std::min(r, sp.var->max_rows);
      sp.rows = std::max(t, r / t * t);
    }
    schedule_all_pairs(sp, sp.tiles_cap);
    sp.kz_max = kz_max_for(ecut, sys[i].L[2]);
    sp.kx_max = kz_max_for(ecut, sys[i].L[0]);
    sp.ky_max = kz_max_for(ecut, sys[i].L[1]);
    sp.psi_off = psi_off;
    sp.m_off = m_off;
    sp.orb_off = orb_off;
    orb_off += sys[i].n_orb;
    psi_off += (long long)sys[i].n_orb * sp.nr;
    m_off += (long long)sys[i].n_orb * sys[i].n_orb;
    // workspace layout of this system
    sp.off_psi32 = off;
    if (precision == HFX_FP32) off = align_up(off + (size_t)sys[i].n_orb * sp.nr * 4);
    sp.nstreams = (sp.batches.size() > 1 && batch_streams == 2) ? 2 : 1;
    sp.off_grids = off;
    sp.grid_bytes = align_up((size_t)sp.slots_per_batch * sp.nr * 2 * elem);
    off = align_up(off + sp.grid_bytes * sp.nstreams);
    sp.off_partials = off;
    {
      // room for every tile pair of the system: a screened schedule (or
      // another virtual group's share) never needs more
      const long long nb = (sys[i].n_orb + sp.var->tile - 1) / sp.var->tile;
      const long long all = nb * (nb + 1) / 2 * bricks_per_tile(sp.var);
      off = align_up(off + (size_t)std::max(sp.n_partials, all) * 8);
    }
    sp.off_gemm = off;
    off = align_up(off + gemm_partial_bytes(sys[i].n_orb, sp.nr));
    sp.off_mean = off;
    if (precision == HFX_FP32) off = align_up(off + (size_t)sys[i].n_orb * sys[i].n_orb * 8);
  }
  // Everything the energy and K psi calls use comes first (all systems);
  // the regions only the other calls use follow.
  p->apply_bytes = off;
  for (int i = 0; i < n_sys; ++i) {
    SystemPlan& sp = p->sys[i];
    sp.off_kpsi = off;
    off = align_up(off + (size_t)sys[i].n_orb * sp.nr * elem);
    sp.off_ortho = off;
    off = align_up(off + (size_t)6 * sys[i].n_orb * sys[i].n_orb * 8 + 64);
    off = align_up(off + (size_t)sys[i].n_orb * std::min<long long>(sp.nr, 32768) * 8);
  }
  p->ws_bytes = off;
  if (ws_cap > 0 && (long long)p->ws_bytes > ws_cap) {
    const size_t need = p->ws_bytes;
    delete p;
    return fail(HFX_ENOMEM, "workspace of " + std::to_string(need) +
                                " bytes exceeds the configured cap " + std::to_string(ws_cap));
  }

  auto cleanup = [&](hfx_status s) {
    for (auto& sp : p->sys) free_system(sp);
    for (auto& st : p->side) (void)hipStreamDestroy(st);
    for (auto& ev : p->join) (void)hipEventDestroy(ev);
    if (p->fork) (void)hipEventDestroy(p->fork);
    delete p;
    return s;
  };
  if (hipGetDevice(&p->device) != hipSuccess)
    return cleanup(fail(HFX_EDEVICE, "no HIP device available"));
  {
    hipError_t e = prepare_apply_left();
    if (e != hipSuccess)
      return cleanup(fail(HFX_EDEVICE, std::string("kernel set-up: ") + hipGetErrorString(e)));
  }
  for (auto& sp : p->sys) {
    hfx_status s;
    if (sp.var->prepare) {
      hipError_t e = sp.var->prepare();
      if (e != hipSuccess)
        return cleanup(fail(HFX_EDEVICE, std::string("kernel set-up: ") + hipGetErrorString(e)));
    }
    // a hybrid mixing fraction scales the kernel, hence E_x, K psi, M and
    // the gradient alike
    sp.v0 = mix * kernel_g0(sp.sys);
    if (precision == HFX_FP64)
      s = upload(kernel_table<double>(sp.sys, false, mix), &sp.vtab);
    else
      s = upload(kernel_table<float>(sp.sys, true, mix), &sp.vtab);
    if (s != HFX_OK) return cleanup(s);
    const Variant* v = sp.var;
    const int* rs[6] = {v->zf, v->zi, v->xf, v->xi, v->yf, v->yi};
    const int cs[6] = {v->nzf, v->nzi, v->nxf, v->nxi, v->nyf, v->nyi};
    for (int k = 0; k < 6; ++k) {
      s = upload_twiddles(rs[k], cs[k], precision, &sp.tw[k]);
      if (s != HFX_OK) return cleanup(s);
    }
    if (v->nzh > 0) {
      s = upload_twiddles(v->zh, v->nzh, precision, &sp.tw[6]);
      if (s != HFX_OK) return cleanup(s);
    }
    void* d = nullptr;
    s = upload(sp.tiles, &d);
    if (s != HFX_OK) return cleanup(s);
    sp.d_tiles = static_cast<TileDesc*>(d);
    s = upload(sp.active, &d);
    if (s != HFX_OK) return cleanup(s);
    sp.d_active = static_cast<int*>(d);
    s = upload(std::vector<double>(kZeroBytes / 8, 0.0), &sp.d_zero);
    if (s != HFX_OK) return cleanup(s);
    if (sp.nstreams == 2) {
      if (hipStreamCreateWithFlags(&sp.bstream, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&sp.ev_fork, hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&sp.ev_join, hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&sp.ev_acc[0], hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&sp.ev_acc[1], hipEventDisableTiming) != hipSuccess)
        return cleanup(fail(HFX_EDEVICE, "stream/event creation failed"));
    }
  }
  if (p->sys.size() > 1) {
    if (hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) != hipSuccess)
      return cleanup(fail(HFX_EDEVICE, "event creation failed"));
    for (size_t i = 0; i < p->sys.size(); ++i) {
      hipStream_t st = nullptr;
      hipEvent_t ev = nullptr;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
        return cleanup(fail(HFX_EDEVICE, "stream/event creation failed"));
      p->side.push_back(st);
      p->join.push_back(ev);
    }
  }
  *out = p;
  for (int i = 0; i < n_sys; ++i)
    log_line("plan system " + std::to_string(i) + ": " + hfx_plan_describe(p, i) +
             " workspace=" + std::to_string(p->ws_bytes));
  return HFX_OK;
}

hfx_status hfx_profile_enable(hfx_plan plan, int enable) {
  if (!plan) return fail(HFX_EINVAL, "null plan");
  plan->prof = enable != 0;
  return HFX_OK;
}

hfx_status hfx_profile_read(hfx_plan plan, double* ms, double* bytes, double* flops,
                            long long* launches, int n) {
  if (!plan) return fail(HFX_EINVAL, "null plan");
  if (n < 0) return fail(HFX_EINVAL, "negative array length");
  for (int k = 0; k < n; ++k) {
    if (ms) ms[k] = 0.0;
    if (bytes) bytes[k] = 0.0;
    if (flops) flops[k] = 0.0;
    if (launches) launches[k] = 0;
  }
  hipError_t err = hipSuccess;
  for (auto& r : plan->recs) {
    float t = 0.f;
    hipError_t e = hipEventSynchronize(r.stop);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.start, r.stop);
    if (e != hipSuccess) err = e;
    if (r.pass < n) {
      if (ms) ms[r.pass] += t;
      if (bytes) bytes[r.pass] += r.bytes;
      if (flops) flops[r.pass] += r.flops;
      if (launches) launches[r.pass] += 1;
    }
    plan->pool.push_back(r.start);
    plan->pool.push_back(r.stop);
  }
  plan->recs.clear();
  if (err != hipSuccess) return fail(HFX_EDEVICE, std::string("event timing: ") + hipGetErrorString(err));
  return HFX_OK;
}

hfx_status hfx_plan_destroy(hfx_plan plan) {
  if (!plan) return fail(HFX_EINVAL, "null plan");
  const hipError_t e = hipDeviceSynchronize();
  for (auto& r : plan->recs) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  for (auto& ev : plan->pool) (void)hipEventDestroy(ev);
  for (auto& st : plan->side) (void)hipStreamDestroy(st);
  for (auto& ev : plan->join) (void)hipEventDestroy(ev);
  if (plan->fork) (void)hipEventDestroy(plan->fork);
  if (plan->cap) (void)hipStreamDestroy(plan->cap);
  for (void* q : plan->retired) (void)hipFree(q);
  for (auto& sp : plan->sys) free_system(sp);
  delete plan;
  if (e != hipSuccess) return fail(HFX_EDEVICE, std::string("pending device error: ") + hipGetErrorString(e));
  return HFX_OK;
}

hfx_status hfx_workspace_size(hfx_plan plan, size_t* bytes) {
  if (!plan) return fail(HFX_EINVAL, "null plan");
  if (!bytes) return fail(HFX_EINVAL, "null output pointer");
  *bytes = plan->ws_bytes;
  return HFX_OK;
}

hfx_status hfx_exchange_energy(hfx_plan plan, const double* psi, double* ex, void* ws,
                               size_t ws_bytes, void* stream) {
  hfx_status s = check_call(plan, psi, ws, ws_bytes);
  if (s != HFX_OK) return s;
  if (!ex) return fail(HFX_EINVAL, "null ex");
  s = check_inputs(plan, psi, static_cast<char*>(ws), static_cast<hipStream_t>(stream));
  if (s != HFX_OK) return s;
  return dispatch_classes(plan, static_cast<hipStream_t>(stream),
                          [&](const std::vector<int>& cls, hipStream_t st) {
                            return enq_energy(plan, cls, psi, ex, static_cast<char*>(ws), st);
                          });
}

hfx_status hfx_apply_exchange(hfx_plan plan, const double* psi, void* kpsi, double* ex,
                              void* ws, size_t ws_bytes, void* stream) {
  hfx_status s = check_call(plan, psi, ws, ws_bytes);
  if (s != HFX_OK) return s;
  if (!kpsi) return fail(HFX_EINVAL, "null kpsi");
  s = check_inputs(plan, psi, static_cast<char*>(ws), static_cast<hipStream_t>(stream));
  if (s != HFX_OK) return s;
  return dispatch_classes(plan, static_cast<hipStream_t>(stream),
                          [&](const std::vector<int>& cls, hipStream_t st) {
                            return enq_apply(plan, cls, psi, kpsi, ex, static_cast<char*>(ws), st);
                          });
}

}  // extern "C"

size_t hfx::apply_workspace_bytes(hfx_plan plan) { return plan->apply_bytes; }

int hfx::plan_device(hfx_plan plan) { return plan->device; }

hfx_status hfx::apply_into(hfx_plan plan, const double* psi, void* kpsi, double* ex, void* ws,
                           void* stream) {
  // the caller checked the arguments and that ws holds apply_workspace_bytes
  plan->quiet = true;
  const hfx_status s = dispatch_classes(
      plan, static_cast<hipStream_t>(stream), [&](const std::vector<int>& cls, hipStream_t st) {
        return enq_apply(plan, cls, psi, kpsi, ex, static_cast<char*>(ws), st);
      });
  plan->quiet = false;
  return s;
}

extern "C" {

hfx_status hfx_exchange_gradient(hfx_plan plan, const double* psi, const double* gscale,
                                 double* grad, void* ws, size_t ws_bytes, void* stream) {
  hfx_status s = check_call(plan, psi, ws, ws_bytes);
  if (s != HFX_OK) return s;
  if (!grad) return fail(HFX_EINVAL, "null grad");
  s = check_inputs(plan, psi, static_cast<char*>(ws), static_cast<hipStream_t>(stream));
  if (s != HFX_OK) return s;
  return dispatch_classes(plan, static_cast<hipStream_t>(stream),
                          [&](const std::vector<int>& cls, hipStream_t st) {
                            return enq_gradient(plan, cls, psi, gscale, grad,
                                                static_cast<char*>(ws), st);
                          });
}

hfx_status hfx_exchange_matrix(hfx_plan plan, const double* psi, double* m, double* ex,
                               void* ws, size_t ws_bytes, void* stream) {
  hfx_status s = check_call(plan, psi, ws, ws_bytes);
  if (s != HFX_OK) return s;
  if (!m) return fail(HFX_EINVAL, "null m");
  s = check_inputs(plan, psi, static_cast<char*>(ws), static_cast<hipStream_t>(stream));
  if (s != HFX_OK) return s;
  return dispatch_classes(plan, static_cast<hipStream_t>(stream),
                          [&](const std::vector<int>& cls, hipStream_t st) {
                            return enq_matrix_full(plan, cls, psi, m, ex,
                                                   static_cast<char*>(ws), st);
                          });
}

hfx_status hfx_exchange_matrix_kpsi(hfx_plan plan, const double* psi, const void* kpsi, double* m,
                                    void* ws, size_t ws_bytes, void* stream) {
  hfx_status s = check_call(plan, psi, ws, ws_bytes);
  if (s != HFX_OK) return s;
  if (!kpsi) return fail(HFX_EINVAL, "null kpsi");
  if (!m) return fail(HFX_EINVAL, "null m");
  return dispatch(plan, static_cast<hipStream_t>(stream), [&](size_t i, hipStream_t st) {
    return enq_matrix(plan, plan->sys[i], psi, kpsi, m, static_cast<char*>(ws), st);
  });
}

hfx_status hfx_orthonormalize(hfx_plan plan, double* psi, int method, void* ws, size_t ws_bytes,
                              void* stream) {
  hfx_status s = check_call(plan, psi, ws, ws_bytes);
  if (s != HFX_OK) return s;
  if (method != HFX_ORTHO_LOWDIN && method != HFX_ORTHO_CHOLESKY)
    return fail(HFX_EINVAL, "unknown orthonormalisation method");
  return dispatch(plan, static_cast<hipStream_t>(stream), [&](size_t i, hipStream_t st) {
    return enq_ortho(plan, plan->sys[i], psi, method, static_cast<char*>(ws), st);
  });
}

hfx_status hfx_ace_build(hfx_plan plan, const void* kpsi, const double* m, double* p, void* ws,
                         size_t ws_bytes, void* stream) {
  g_last_error.clear();
  hfx_status s = check_call(plan, kpsi, ws, ws_bytes);
  if (s != HFX_OK) return s;
  if (!m) return fail(HFX_EINVAL, "null m");
  if (!p) return fail(HFX_EINVAL, "null p");
  return dispatch(plan, static_cast<hipStream_t>(stream), [&](size_t i, hipStream_t st) {
    return enq_ace_build(plan, plan->sys[i], kpsi, m, p, static_cast<char*>(ws), st);
  });
}

hfx_status hfx_ace_apply(hfx_plan plan, const double* p, const double* phi, double* out,
                         void* ws, size_t ws_bytes, void* stream) {
  g_last_error.clear();
  hfx_status s = check_call(plan, p, ws, ws_bytes);
  if (s != HFX_OK) return s;
  if (!phi) return fail(HFX_EINVAL, "null phi");
  if (!out) return fail(HFX_EINVAL, "null out");
  if (out == p || out == phi) return fail(HFX_EINVAL, "out must not alias p or phi");
  return dispatch(plan, static_cast<hipStream_t>(stream), [&](size_t i, hipStream_t st) {
    return enq_ace_apply(plan, plan->sys[i], p, phi, out, static_cast<char*>(ws), st);
  });
}

// s-MTACE pair screening: keep pairs with int |psi_a psi_b| dV >= rho_cut and
// rebuild the tile schedule of every system over them.
hfx_status hfx_screen(hfx_plan plan, const double* psi, double rho_cut, long long* kept, void* ws,
                      size_t ws_bytes, void* stream) {
  g_last_error.clear();
  hfx_status s = check_call(plan, psi, ws, ws_bytes);
  if (s != HFX_OK) return s;
  if (!std::isfinite(rho_cut)) return fail(HFX_EINVAL, "rho_cut must be finite");
  if (plan->capturing) return fail(HFX_EINVAL, "hfx_screen cannot be captured");
  for (const SystemPlan& sp : plan->sys)
    if (sp.var->tile != 8) return fail(HFX_EUNSUPPORTED, "screening needs 8-orbital tiles");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  for (size_t i = 0; i < plan->sys.size(); ++i) {
    SystemPlan& sp = plan->sys[i];
    const int n = sp.sys.n_orb;
    std::vector<unsigned char> keep((size_t)n * n, 1);
    std::vector<int> perm(n);
    for (int k = 0; k < n; ++k) perm[k] = k;
    const bool screened = rho_cut > 0.0;
    if (screened) {
      double* part = reinterpret_cast<double*>(w + sp.off_gemm);
      double* amat = reinterpret_cast<double*>(w + sp.off_ortho);
      launch_xtx_abs(psi + sp.psi_off, n, sp.nr, sp.dv, part, amat, st);
      HIP_TRY(hipGetLastError());
      std::vector<double> h((size_t)n * n);
      HIP_TRY(hipMemcpyAsync(h.data(), amat, h.size() * 8, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      // A is symmetric up to rounding: take the upper triangle, so that each
      // unordered pair is decided once
      for (int a = 0; a < n; ++a)
        for (int b = a; b < n; ++b) {
          h[(size_t)b * n + a] = h[(size_t)a * n + b];
          const unsigned char k = h[(size_t)a * n + b] >= rho_cut ? 1 : 0;
          keep[(size_t)a * n + b] = keep[(size_t)b * n + a] = k;
        }
      perm = cluster_order(n, sp.var->tile, h, keep);
    } else {
      HIP_TRY(hipStreamSynchronize(st));
    }
    if (kept) {
      long long c = 0;
      for (int a = 0; a < n; ++a)
        for (int b = a; b < n; ++b) c += keep[(size_t)a * n + b];
      kept[i] = c;
    }
    // The new schedule goes into a copy; the plan keeps its old schedule and
    // tables until every new table is on the device.
    SystemPlan ns = sp;
    if (screened)
      schedule_kept_pairs(ns, keep, perm);
    else
      schedule_all_pairs(ns, sp.tiles_cap);
    void *dt = nullptr, *da = nullptr, *dp = nullptr, *dk = nullptr;
    if ((s = upload(ns.tiles, &dt)) != HFX_OK || (s = upload(ns.active, &da)) != HFX_OK ||
        (screened && ((s = upload(perm, &dp)) != HFX_OK || (s = upload(keep, &dk)) != HFX_OK))) {
      for (void* q : {dt, da, dp, dk})
        if (q) (void)hipFree(q);
      return s;
    }
    // The stream is idle (synchronised above).  Graphs captured earlier
    // still read the old tables: retire them while any graph is alive.
    for (void* q : {(void*)sp.d_tiles, (void*)sp.d_active, (void*)sp.d_perm, (void*)sp.d_keep}) {
      if (!q) continue;
      if (plan->live_graphs > 0)
        plan->retired.push_back(q);
      else
        (void)hipFree(q);
    }
    sp.tiles = std::move(ns.tiles);
    sp.active = std::move(ns.active);
    sp.batches = std::move(ns.batches);
    sp.n_partials = ns.n_partials;
    sp.tiles_per_batch = ns.tiles_per_batch;
    sp.slots_per_batch = ns.slots_per_batch;
    sp.d_tiles = static_cast<TileDesc*>(dt);
    sp.d_active = static_cast<int*>(da);
    sp.d_perm = static_cast<int*>(dp);
    sp.d_keep = static_cast<unsigned char*>(dk);
  }
  return HFX_OK;
}

const char* hfx_plan_describe(hfx_plan plan, int system) {
  if (!plan || system < 0 || system >= (int)plan->sys.size()) {
    (void)fail(HFX_EINVAL, "null plan or no such system");
    return nullptr;
  }
  const SystemPlan& sp = plan->sys[system];
  const Variant* v = sp.var;
  auto sched = [](const int* r, int c) {
    std::string o;
    for (int i = 0; i < c; ++i) o += (i ? "x" : "") + std::to_string(r[i]);
    return o;
  };
  std::string d = std::string("variant=") + v->name + " n=" + std::to_string(v->n) +
                  (v->nz != v->n ? " nz=" + std::to_string(v->nz) : std::string()) +
                  " tile=" + std::to_string(v->tile) + " brick=" + std::to_string(v->brick) +
                  " z=" + sched(v->zf, v->nzf) + "/" + sched(v->zi, v->nzi) +
                  " x=" + sched(v->xf, v->nxf) + "/" + sched(v->xi, v->nxi) +
                  " y=" + sched(v->yf, v->nyf) + "/" + sched(v->yi, v->nyi) +
                  " threads=" + std::to_string(v->nt_fwd) + "/" +
                  std::to_string(v->plane_mode == 0 ? v->nt_plane : v->nt_cols) + "/" +
                  std::to_string(v->nt_acc) + " plane=" +
                  (v->plane_mode == 0 ? "fused" : "split") +
                  " rows=" + std::to_string(sp.rows) +
                  (sp.kz_max < v->nz / 2 ? " kz_max=" + std::to_string(sp.kz_max)
                                          : std::string()) +
                  (half_z(v, sp.kz_max) ? " z_fwd=half(" + sched(v->zh, v->nzh) + ")"
                                        : std::string()) +
                  (half_y(v, sp.kx_max, sp.ky_max) ? " y_rows=half" : std::string()) +
                  (half_x(v, sp.kx_max, sp.ky_max) ? " x_cols=half" : std::string()) +
                  " tiles_per_batch=" + std::to_string(sp.tiles_per_batch) +
                  " batches=" + std::to_string(sp.batches.size()) +
                  " streams=" + std::to_string(sp.nstreams) +
                  " screened=" + (sp.d_keep ? "yes" : "no") +
                  " tuned=" + (sp.tuned ? "yes" : "no");
  {
    // the size class: systems that share the pass launches of exchange calls
    const std::vector<std::vector<int>> cls = size_classes(plan);
    for (size_t c = 0; c < cls.size(); ++c)
      for (int i : cls[c])
        if (i == system)
          d += " class=" + std::to_string(c) + "/" + std::to_string(cls[c].size());
  }
  plan->desc = d;
  return plan->desc.c_str();
}

hfx_status hfx_scdm(hfx_plan plan, const double* psi, double* phi, int* pivots, void* ws,
                    size_t ws_bytes, void* stream) {
  g_last_error.clear();
  hfx_status s = check_call(plan, psi, ws, ws_bytes);
  if (s != HFX_OK) return s;
  if (!phi) return fail(HFX_EINVAL, "null phi");
  if (plan->capturing) return fail(HFX_EINVAL, "hfx_scdm cannot be captured");
  for (const SystemPlan& sp : plan->sys) {
    // the pivot step keeps two n-vectors in LDS
    if (sp.sys.n_orb > 3500) return fail(HFX_EUNSUPPORTED, "hfx_scdm supports up to 3500 orbitals");
    if (sp.sys.n_orb > sp.nr) return fail(HFX_EINVAL, "more orbitals than grid points");
  }
  return dispatch(plan, static_cast<hipStream_t>(stream), [&](size_t i, hipStream_t st) {
    return enq_scdm(plan, plan->sys[i], psi, phi, pivots, static_cast<char*>(ws), st);
  });
}

hfx_status hfx_schedule_info(hfx_plan plan, int system, long long* info) {
  if (!plan) return fail(HFX_EINVAL, "null plan");
  if (!info) return fail(HFX_EINVAL, "null info");
  if (system < 0 || system >= (int)plan->sys.size()) return fail(HFX_EINVAL, "no such system");
  const SystemPlan& sp = plan->sys[system];
  long long pairs = 0;
  const bool masked = sp.d_keep != nullptr;  // screened schedules carry pair masks
  for (const TileDesc& td : sp.tiles)
    for (int a = 0; a < td.nI; ++a)
      for (int b = 0; b < td.nJ; ++b)
        if (!(td.diag && b + td.joff < a) && (!masked || keep_bit(td, a, b))) ++pairs;
  info[0] = (long long)sp.batches.size();
  info[1] = (long long)sp.tiles.size();
  info[2] = (long long)sp.active.size();
  info[3] = pairs;
  return HFX_OK;
}

hfx_status hfx_graph_create(hfx_plan plan, int op, double* psi, void* kpsi, double* ex,
                            double* m, void* ws, size_t ws_bytes, hfx_graph* out) {
  if (!out) return fail(HFX_EINVAL, "null output graph pointer");
  *out = nullptr;
  hfx_status s = check_call(plan, psi, ws, ws_bytes);
  if (s != HFX_OK) return s;
  if (op != HFX_GRAPH_ENERGY && op != HFX_GRAPH_APPLY && op != HFX_GRAPH_STEP)
    return fail(HFX_EINVAL, "unknown graph operation");
  if (op == HFX_GRAPH_ENERGY && !ex) return fail(HFX_EINVAL, "null ex");
  if (op != HFX_GRAPH_ENERGY && !kpsi) return fail(HFX_EINVAL, "null kpsi");
  if (op == HFX_GRAPH_STEP && !m) return fail(HFX_EINVAL, "null m");
  if (!plan->cap) HIP_TRY(hipStreamCreateWithFlags(&plan->cap, hipStreamNonBlocking));
  hfx_graph g = new hfx_graph_t();
  g->plan = plan;
  plan->capturing = true;
  hipError_t e = hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    plan->capturing = false;
    delete g;
    return fail(HFX_EDEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  }
  char* w = static_cast<char*>(ws);
  s = dispatch_classes(plan, plan->cap, [&](const std::vector<int>& cls, hipStream_t st) {
    hfx_status r = HFX_OK;
    if (op == HFX_GRAPH_ENERGY) return enq_energy(plan, cls, psi, ex, w, st);
    if (op == HFX_GRAPH_STEP)
      for (int i : cls)
        if (r == HFX_OK) r = enq_ortho(plan, plan->sys[i], psi, HFX_ORTHO_LOWDIN, w, st);
    if (r == HFX_OK) r = enq_apply(plan, cls, psi, kpsi, ex, w, st);
    if (op == HFX_GRAPH_STEP)
      for (int i : cls)
        if (r == HFX_OK) r = enq_matrix(plan, plan->sys[i], psi, kpsi, m, w, st);
    return r;
  });
  e = hipStreamEndCapture(plan->cap, &g->graph);
  plan->capturing = false;
  if (s != HFX_OK || e != hipSuccess) {
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    if (s != HFX_OK) return s;
    return fail(HFX_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  }
  e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g->graph);
    delete g;
    return fail(HFX_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  ++plan->live_graphs;
  *out = g;
  return HFX_OK;
}

hfx_status hfx_graph_launch(hfx_graph g, void* stream) {
  if (!g || !g->exec) return fail(HFX_EINVAL, "null graph");
  HIP_TRY(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
  return HFX_OK;
}

hfx_status hfx_graph_destroy(hfx_graph g) {
  if (!g) return fail(HFX_EINVAL, "null graph");
  hipError_t e = hipSuccess;
  if (g->exec) e = hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  hfx_plan plan = g->plan;
  delete g;
  if (plan && --plan->live_graphs == 0 && !plan->retired.empty()) {
    // the last graph that could read the retired tables is gone; a replay
    // still in flight may read them, so wait for the device first
    const hipError_t w = hipDeviceSynchronize();
    if (e == hipSuccess) e = w;
    for (void* q : plan->retired) (void)hipFree(q);
    plan->retired.clear();
  }
  if (e != hipSuccess) return fail(HFX_EDEVICE, std::string("hipGraphExecDestroy: ") + hipGetErrorString(e));
  return HFX_OK;
}

}  // extern "C"
