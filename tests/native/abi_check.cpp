// Host checks of the C ABI's argument handling, run on the CPU (no GPU) in a
// build whose host code carries AddressSanitizer and UndefinedBehaviorSanitizer:
// option parsing (per-system lists, every key, malformed values), validation
// of systems, the clean-up path of a plan whose device set-up fails, the
// tune-cache file helpers, the autotuner's argument errors and every entry
// point's null-plan path.  Prints ALL OK and exits 0 when every check holds;
// a sanitizer report aborts the run.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "../../include/hfx.h"
#include "../../paper_2309_00651_amd/csrc/tune.hpp"

static int g_fail = 0, g_checks = 0;
#define CHECK(c)                                              \
  do {                                                        \
    ++g_checks;                                               \
    if (!(c)) {                                               \
      std::printf("FAIL line %d: %s\n", __LINE__, #c);        \
      ++g_fail;                                               \
    }                                                         \
  } while (0)

static hfx_system sys(int n, int nz, double L, int n_orb, int kernel = 0, double w = 0.0) {
  hfx_system s;
  s.n[0] = s.n[1] = n;
  s.n[2] = nz;
  s.L[0] = s.L[1] = L;
  s.L[2] = L * nz / n;
  s.n_orb = n_orb;
  s.kernel = kernel;
  s.param = w;
  return s;
}

static hfx_status create(const hfx_system* s, int n, int prec, const char* opts) {
  hfx_plan p = nullptr;
  const hfx_status st = hfx_plan_create(&p, s, n, prec, opts);
  if (st == HFX_OK) hfx_plan_destroy(p);  // only with a device
  else CHECK(p == nullptr);
  return st;
}

int main() {
  for (int c = 0; c < 5; ++c) CHECK(std::strncmp(hfx_status_string((hfx_status)c), "HFX_", 4) == 0);
  for (int n : {24, 64, 72, 80, 96, 108, 120, 128})
    for (int prec : {0, 1}) CHECK(std::strlen(hfx_variants(n, prec)) > 0);
  CHECK(std::strlen(hfx_variants(50, 0)) == 0);

  const hfx_system good = sys(24, 24, 10.0, 8);
  const hfx_system two[2] = {sys(24, 24, 10.0, 9), sys(64, 64, 12.0, 13, 1, 0.106)};
  // malformed options: rejected before any device call
  const char* bad[] = {"tiles=", "tiles=-1", "tiles=x", "rows=12", "rows=64", "rows=", "mix=0",
                       "mix=2", "mix=", "ecut=-1", "ecut=", "ecut=1e9", "streams=3", "shard=1",
                       "shard=3/2", "variant=nope", "bogus=1", "tiles", "check=2", "check=",
                       "tune_cache=", "maxws=abc", "rows=8,16", "variant=a,b"};
  for (const char* o : bad) {
    const hfx_status st = create(&good, 1, 0, o);
    CHECK(st == HFX_EINVAL);
    CHECK(std::strlen(hfx_last_error()) > 0);
  }
  for (const char* o : {"rows=8,16,32", "tiles=1,2,3", "variant=f32-n24", "tiles=4,x"})
    CHECK(create(two, 2, 0, o) == HFX_EINVAL);
  CHECK(create(two, 2, 1, "variant=f32-n24,f32-n64") == HFX_EINVAL);  // float32 names, float64 plan
  // invalid systems
  hfx_system s = good;
  s.n_orb = 0;
  CHECK(create(&s, 1, 0, nullptr) == HFX_EINVAL);
  s = good;
  s.L[1] = -1.0;
  CHECK(create(&s, 1, 0, nullptr) == HFX_EINVAL);
  s = good;
  s.kernel = 1;
  s.param = 0.0;
  CHECK(create(&s, 1, 0, nullptr) == HFX_EINVAL);
  s = good;
  s.n[1] = 32;
  CHECK(create(&s, 1, 0, nullptr) == HFX_EUNSUPPORTED);
  s = sys(50, 50, 10.0, 4);
  CHECK(create(&s, 1, 0, nullptr) == HFX_EUNSUPPORTED);
  CHECK(create(&good, 0, 0, nullptr) == HFX_EINVAL);
  CHECK(create(&good, 1, 7, nullptr) == HFX_EINVAL);
  CHECK(hfx_plan_create(nullptr, &good, 1, 0, nullptr) == HFX_EINVAL);
  // valid options: every parse succeeds; without a device the set-up fails
  // cleanly (or succeeds where a device exists)
  for (const char* o : {(const char*)nullptr, "tiles=2;rows=16;ecut=5;mix=0.25;check=1",
                        "variant=f32-n24;streams=2;shard=1/3", "maxws=1000000000000"}) {
    const hfx_status st = create(&good, 1, 0, o);
    CHECK(st == HFX_OK || st == HFX_EDEVICE);
  }
  {
    const hfx_status st = create(two, 2, 0, "variant=f32-n24,f32-n64-r;rows=8,16;tiles=0,3");
    CHECK(st == HFX_OK || st == HFX_EDEVICE);
  }
  // tune cache helpers
  {
    char path[] = "/tmp/hfx_tune_checkXXXXXX";
    const int fd = mkstemp(path);
    CHECK(fd >= 0);
    std::string o;
    CHECK(!hfx::tune_lookup(path, "k1", &o));
    CHECK(hfx::tune_store(path, "k1", "variant=a;tiles=0;rows=8", 1.5, {{"c1", 1.5}, {"c2", 2.0}}));
    CHECK(hfx::tune_store(path, "k2", "variant=b;tiles=4;rows=16", 2.5, {}));
    CHECK(hfx::tune_store(path, "k1", "variant=c;tiles=0;rows=32", 1.25, {{"c3", 1.25}}));
    CHECK(hfx::tune_lookup(path, "k1", &o) && o == "variant=c;tiles=0;rows=32");
    CHECK(hfx::tune_lookup(path, "k2", &o) && o == "variant=b;tiles=4;rows=16");
    CHECK(!hfx::tune_lookup(path, "k1#candidate", &o) || o == "c3");
    CHECK(!hfx::tune_lookup("/nonexistent/dir/cache", "k1", &o));
    CHECK(!hfx::tune_store("/nonexistent/dir/cache", "k1", "x", 1.0, {}));
    std::remove(path);
    CHECK(hfx::kz_max_for(0.0, 10.0) > 1000);
    CHECK(hfx::kz_max_for(5.0, 10.0) == 2 * 5);  // sqrt(10) 10 / 2 pi = 5.03
    const std::string key = hfx::tune_key(good, 0, hfx::kz_max_for(0.0, 10.0), "gfx950");
    CHECK(key.find("n=24x24x24") != std::string::npos && key.find("kz_max=-1") != std::string::npos);
  }
  // autotuner argument errors
  {
    char buf[64];
    const double* fake = reinterpret_cast<const double*>(&good);
    CHECK(hfx_autotune(nullptr, 1, 0, nullptr, fake, 1, nullptr, buf, 64, nullptr) == HFX_EINVAL);
    CHECK(hfx_autotune(&good, 0, 0, nullptr, fake, 1, nullptr, buf, 64, nullptr) == HFX_EINVAL);
    CHECK(hfx_autotune(&good, 1, 0, nullptr, nullptr, 1, nullptr, buf, 64, nullptr) == HFX_EINVAL);
    CHECK(hfx_autotune(&good, 1, 3, nullptr, fake, 1, nullptr, buf, 64, nullptr) == HFX_EINVAL);
    CHECK(hfx_autotune(&good, 1, 0, "ecut=5;rows=8", fake, 1, nullptr, buf, 64, nullptr) ==
          HFX_EINVAL);
  }
  // every entry point's null-plan path
  void* d = reinterpret_cast<void*>(256);
  double* dd = reinterpret_cast<double*>(256);
  CHECK(hfx_plan_destroy(nullptr) == HFX_EINVAL);
  size_t ws = 0;
  CHECK(hfx_workspace_size(nullptr, &ws) == HFX_EINVAL);
  CHECK(hfx_exchange_energy(nullptr, dd, dd, d, 0, nullptr) == HFX_EINVAL);
  CHECK(hfx_apply_exchange(nullptr, dd, d, dd, d, 0, nullptr) == HFX_EINVAL);
  CHECK(hfx_exchange_matrix(nullptr, dd, dd, nullptr, d, 0, nullptr) == HFX_EINVAL);
  CHECK(hfx_exchange_matrix_kpsi(nullptr, dd, d, dd, d, 0, nullptr) == HFX_EINVAL);
  CHECK(hfx_exchange_gradient(nullptr, dd, nullptr, dd, d, 0, nullptr) == HFX_EINVAL);
  CHECK(hfx_orthonormalize(nullptr, dd, 0, d, 0, nullptr) == HFX_EINVAL);
  CHECK(hfx_ace_build(nullptr, d, dd, dd, d, 0, nullptr) == HFX_EINVAL);
  CHECK(hfx_ace_apply(nullptr, dd, dd, dd, d, 0, nullptr) == HFX_EINVAL);
  CHECK(hfx_screen(nullptr, dd, 1e-3, nullptr, d, 0, nullptr) == HFX_EINVAL);
  CHECK(hfx_scdm(nullptr, dd, dd, nullptr, d, 0, nullptr) == HFX_EINVAL);
  long long info[4];
  CHECK(hfx_schedule_info(nullptr, 0, info) == HFX_EINVAL);
  CHECK(hfx_plan_describe(nullptr, 0) == nullptr);
  CHECK(hfx_profile_enable(nullptr, 1) == HFX_EINVAL);
  CHECK(hfx_graph_launch(nullptr, nullptr) == HFX_EINVAL);
  CHECK(hfx_graph_destroy(nullptr) == HFX_EINVAL);
  std::printf("%d checks, %d failures\n", g_checks, g_fail);
  if (g_fail == 0) std::printf("ALL OK\n");
  return g_fail == 0 ? 0 : 1;
}
