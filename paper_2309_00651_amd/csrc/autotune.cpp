// Autotuner and tune cache (host code).
//
// hfx_autotune times every compiled kernel configuration of a system's grid
// (variants: radix orders, plane threads, psi staging) crossed with the
// batch size (tiles per batch: the default, or 4) and the rows per tile pair
// (8, 16, 32, up to the orbital count) on the caller's orbitals, with HIP
// events around hfx_apply_exchange, and keeps the fastest.  Among the
// candidates within 5 % of the fastest the first in a fixed order wins, the
// plan defaults coming first: configurations closer than that differ by
// about the run-to-run spread of the same launches (1-3 % measured on one
// MI355X), so a narrower window lets timing noise flip the choice.  Choices are cached in a text file, one line per
// key: "<key> <options> <ms>"; plan creation reads them back (option
// tune_cache= or the environment variable HFX_AUTOTUNE_CACHE).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/hfx.h"
#include "hfx_internal.hpp"
#include "tune.hpp"

#ifndef HFX_SOURCES_ID
#define HFX_SOURCES_ID "unversioned"
#endif

namespace hfx {

int kz_max_for(double ecut, double lz) {
  if (!(ecut > 0.0)) return 1 << 30;
  const double mz = std::sqrt(2.0 * ecut) * lz / (2.0 * 3.14159265358979323846);
  return 2 * (int)std::floor(mz + 1e-9);
}

std::string device_arch(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

const char* build_id() { return HFX_SOURCES_ID; }

std::string tune_key(const hfx_system& s, int precision, int kz_max, const std::string& arch) {
  // kz_max beyond the grid means no band limit
  const int kz = kz_max >= s.n[2] / 2 ? -1 : kz_max;
  return "arch=" + arch + "|n=" + std::to_string(s.n[0]) + "x" + std::to_string(s.n[1]) + "x" +
         std::to_string(s.n[2]) + "|n_orb=" + std::to_string(s.n_orb) +
         "|prec=" + std::to_string(precision) + "|kz_max=" + std::to_string(kz) +
         "|build=" + build_id();
}

bool tune_lookup(const std::string& path, const std::string& key, std::string* options) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream ls(line);
    std::string k, o;
    if (ls >> k >> o && k == key) {
      *options = o;
      return true;
    }
  }
  return false;
}

bool tune_store(const std::string& path, const std::string& key, const std::string& options,
                double ms, const std::vector<std::pair<std::string, double>>& timings) {
  // the key's choice and its candidate table replace earlier ones
  const std::string table = key + "#candidate";
  std::vector<std::string> lines;
  {
    std::ifstream f(path);
    std::string line;
    while (f && std::getline(f, line)) {
      std::istringstream ls(line);
      std::string k;
      if (ls >> k && k != key && k != table) lines.push_back(line);
    }
  }
  char buf[64];
  std::snprintf(buf, sizeof buf, "%.4f", ms);
  lines.push_back(key + " " + options + " " + buf);
  for (const auto& t : timings) {
    std::snprintf(buf, sizeof buf, "%.4f", t.second);
    lines.push_back(table + " " + t.first + " " + buf);
  }
  const std::string tmp = path + ".tmp";
  {
    std::ofstream o(tmp, std::ios::trunc);
    if (!o) return false;
    for (const std::string& l : lines) o << l << "\n";
    if (!o) return false;
  }
  return std::rename(tmp.c_str(), path.c_str()) == 0;
}

}  // namespace hfx

namespace {

// Candidates this much slower than the fastest still count as ties.
constexpr double kTieWindow = 0.05;

struct DeviceBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t want) {
    if (want <= bytes) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    const hipError_t e = hipMalloc(&p, want ? want : 1);
    if (e == hipSuccess) bytes = want;
    return e;
  }
  ~DeviceBuf() {
    if (p) (void)hipFree(p);
  }
};

// Time one candidate: the fastest of reps applies, each bracketed by its own
// events, after one warm-up (the minimum is the least noisy estimate of a
// kernel sequence's cost); ms per apply, < 0 on failure (status in *st).
double time_candidate(const hfx_system& s, int prec, const std::string& opts, const double* psi,
                      int reps, DeviceBuf& ws, DeviceBuf& kpsi, DeviceBuf& ex, hipStream_t st,
                      hfx_status* status) {
  hfx_plan p = nullptr;
  *status = hfx_plan_create(&p, &s, 1, prec, opts.c_str());
  if (*status != HFX_OK) return -1.0;
  size_t wb = 0;
  (void)hfx_workspace_size(p, &wb);
  double ms = -1.0;
  hipEvent_t a = nullptr, b = nullptr;
  if (ws.ensure(wb) != hipSuccess || hipEventCreate(&a) != hipSuccess ||
      hipEventCreate(&b) != hipSuccess) {
    *status = HFX_ENOMEM;
  } else {
    *status = hfx_apply_exchange(p, psi, kpsi.p, static_cast<double*>(ex.p), ws.p, ws.bytes, st);
    for (int r = 0; r < reps && *status == HFX_OK; ++r) {
      if (hipEventRecord(a, st) != hipSuccess) {
        *status = HFX_EDEVICE;
        break;
      }
      *status = hfx_apply_exchange(p, psi, kpsi.p, static_cast<double*>(ex.p), ws.p, ws.bytes, st);
      float t = 0.f;
      if (*status == HFX_OK && (hipEventRecord(b, st) != hipSuccess ||
                                hipEventSynchronize(b) != hipSuccess ||
                                hipEventElapsedTime(&t, a, b) != hipSuccess))
        *status = HFX_EDEVICE;
      if (*status == HFX_OK && (ms < 0.0 || t < ms)) ms = t;
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hfx_plan_destroy(p);
  return ms;
}

}  // namespace

extern "C" hfx_status hfx_autotune(const hfx_system* sys, int n_sys, int precision,
                                   const char* options, const double* psi, int reps,
                                   const char* cache_path, char* chosen_host, size_t chosen_bytes,
                                   void* stream) {
  using namespace hfx;
  if (!sys || n_sys < 1 || !psi) {
    set_error("null system array or psi, or n_sys < 1");
    return HFX_EINVAL;
  }
  if (precision != HFX_FP32 && precision != HFX_FP64) {
    set_error("precision must be HFX_FP32 or HFX_FP64");
    return HFX_EINVAL;
  }
  const std::string base = options ? options : "";
  for (const char* k : {"variant=", "tiles=", "rows=", "tune_cache="})
    if (base.find(k) != std::string::npos) {
      set_error(std::string("the autotuner chooses ") + k + " itself");
      return HFX_EINVAL;
    }
  if (reps < 1) reps = 2;
  double ecut = 0.0;
  {
    const size_t e = base.find("ecut=");
    if (e != std::string::npos) ecut = std::strtod(base.c_str() + e + 5, nullptr);
  }
  const hipStream_t st = static_cast<hipStream_t>(stream);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    set_error("no HIP device");
    return HFX_EDEVICE;
  }
  const std::string arch = device_arch(dev);
  const size_t elem = precision == HFX_FP64 ? 8 : 4;
  std::vector<std::string> cv(n_sys), ct(n_sys), cr(n_sys);
  DeviceBuf ws, kpsi, ex;
  if (ex.ensure(8) != hipSuccess) {
    set_error("device allocation failed");
    return HFX_ENOMEM;
  }
  long long off = 0;
  for (int i = 0; i < n_sys; ++i) {
    const hfx_system& s = sys[i];
    const long long nr = (long long)s.n[0] * s.n[1] * s.n[2];
    const double* ps = psi + off;
    off += (long long)s.n_orb * nr;
    const std::string key = tune_key(s, precision, kz_max_for(ecut, s.L[2]), arch);
    std::string best;
    if (cache_path && tune_lookup(cache_path, key, &best)) {
      // cached choice: nothing to time
    } else {
      int count = 0;
      const Variant* vs = precision == HFX_FP64 ? variants_f64(&count) : variants_f32(&count);
      const int drows = default_rows(s.n_orb);
      const int rmax = (s.n_orb + 7) / 8 * 8;
      std::vector<int> rows_order = {drows};
      for (int r : {8, 16, 32})
        if (r != drows) rows_order.push_back(r);
      std::vector<std::string> cands;
      for (int v = 0; v < count; ++v) {
        if (vs[v].n != s.n[0] || vs[v].nz != s.n[2]) continue;
        for (int t : {0, 4})
          for (int r : rows_order) {
            if (r > vs[v].max_rows || (r > rmax && r != 8)) continue;
            cands.push_back(std::string("variant=") + vs[v].name + ";tiles=" +
                            std::to_string(t) + ";rows=" + std::to_string(r));
          }
      }
      if (cands.empty()) {
        set_error("no compiled configuration for the grid of system " + std::to_string(i));
        return HFX_EUNSUPPORTED;
      }
      if (kpsi.ensure((size_t)s.n_orb * nr * elem) != hipSuccess) {
        set_error("device allocation failed");
        return HFX_ENOMEM;
      }
      std::vector<double> ms(cands.size(), -1.0);
      double fastest = 0.0;
      {
        // bring the device to its working clocks and load the kernels
        hfx_status status = HFX_OK;
        const std::string opts = base.empty() ? cands[0] : base + ";" + cands[0];
        (void)time_candidate(s, precision, opts, ps, 2, ws, kpsi, ex, st, &status);
      }
      for (size_t c = 0; c < cands.size(); ++c) {
        hfx_status status = HFX_OK;
        const std::string opts = base.empty() ? cands[c] : base + ";" + cands[c];
        ms[c] = time_candidate(s, precision, opts, ps, reps, ws, kpsi, ex, st, &status);
        if (status == HFX_ENOMEM) continue;  // a candidate's workspace that does not fit
        if (status != HFX_OK) {
          set_error("candidate " + opts + " failed: " + hfx_last_error());
          return status;
        }
        if (fastest <= 0.0 || ms[c] < fastest) fastest = ms[c];
        log_line("autotune system " + std::to_string(i) + ": " + opts + " " +
                 std::to_string(ms[c]) + " ms");
      }
      if (!(fastest > 0.0)) {
        set_error("no candidate could be timed for system " + std::to_string(i));
        return HFX_ENOMEM;
      }
      size_t pick = 0;
      while (!(ms[pick] > 0.0 && ms[pick] <= fastest * (1.0 + kTieWindow))) ++pick;
      best = cands[pick];
      log_line("autotune system " + std::to_string(i) + ": chose " + best);
      std::vector<std::pair<std::string, double>> table;
      for (size_t c = 0; c < cands.size(); ++c)
        if (ms[c] > 0.0) table.emplace_back(cands[c], ms[c]);
      if (cache_path && !tune_store(cache_path, key, best, ms[pick], table)) {
        set_error(std::string("cannot write the tune cache ") + cache_path);
        return HFX_EINVAL;
      }
    }
    // split "variant=..;tiles=..;rows=.." into the per-system lists
    std::istringstream is(best);
    std::string item;
    while (std::getline(is, item, ';')) {
      if (item.rfind("variant=", 0) == 0) cv[i] = item.substr(8);
      if (item.rfind("tiles=", 0) == 0) ct[i] = item.substr(6);
      if (item.rfind("rows=", 0) == 0) cr[i] = item.substr(5);
    }
  }
  if (chosen_host) {
    std::string out;
    auto join = [&](const char* k, const std::vector<std::string>& v) {
      out += (out.empty() ? "" : ";") + std::string(k) + "=";
      for (int i = 0; i < n_sys; ++i) out += (i ? "," : "") + v[i];
    };
    join("variant", cv);
    join("tiles", ct);
    join("rows", cr);
    if (out.size() + 1 > chosen_bytes) {
      set_error("chosen_host holds " + std::to_string(chosen_bytes) + " bytes, " +
              std::to_string(out.size() + 1) + " needed");
      return HFX_EINVAL;
    }
    std::memcpy(chosen_host, out.c_str(), out.size() + 1);
  }
  return HFX_OK;
}
