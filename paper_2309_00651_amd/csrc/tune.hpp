// Host-side helpers shared by the plan (hfx_api.cpp), the autotuner
// (autotune.cpp) and the entry point that allocates nothing (noalloc.hip).
#pragma once

#include <string>
#include <utility>
#include <vector>

#include "../../include/hfx.h"

namespace hfx {

// kz band of the pair densities of orbitals inside the plane-wave sphere
// (1/2)|G|^2 <= ecut on a box of length lz along z: orbitals have
// |m_z| <= sqrt(2 ecut) lz / (2 pi), their products twice that.  ecut <= 0:
// no band limit (a value above any grid's n_z / 2).
int kz_max_for(double ecut, double lz);

// Architecture name of a HIP device ("gfx950"), without target features.
std::string device_arch(int device);

// Cache key of one system: device architecture, grid, orbital count,
// precision, kz band and the identity of the compiled kernel sources.  The
// box lengths and the kernel kind do not change the work and are not part
// of it.
std::string tune_key(const hfx_system& s, int precision, int kz_max, const std::string& arch);

// Options stored for key in the cache file at path ("variant=..;tiles=..;
// rows=.."); false when the file or the key is missing.
bool tune_lookup(const std::string& path, const std::string& key, std::string* options);

// Adds or replaces the line of key and its candidate table (one line
// "<key>#candidate <options> <ms>" per timed candidate), written to a
// temporary file that is then renamed over the cache.  False when the file
// cannot be written.
bool tune_store(const std::string& path, const std::string& key, const std::string& options,
                double ms, const std::vector<std::pair<std::string, double>>& timings);

// Identity of the kernel sources the library was built from.
const char* build_id();

// Rows per tile pair of a plan that names none (hfx_api.cpp).
int default_rows(int n_orb);

// Sets the thread-local text hfx_last_error() returns (hfx_api.cpp).
void set_error(const std::string& msg);

// Leading workspace bytes the energy and K psi calls of a plan use, the
// plan's device, and hfx_apply_exchange's launch sequence on a workspace of
// that size with no profiling events (hfx_api.cpp).
size_t apply_workspace_bytes(hfx_plan plan);
int plan_device(hfx_plan plan);
hfx_status apply_into(hfx_plan plan, const double* psi, void* kpsi, double* ex, void* ws,
                      void* stream);

// One line "[hfx] msg" on stderr when the environment variable HFX_LOG is set
// to a non-empty value other than "0" (hfx_api.cpp).
void log_line(const std::string& msg);

}  // namespace hfx
