// Host LAPACK, resolved at run time.
//
// The library itself links no LAPACK.  The FP64 eigendecomposition of the
// seed (Section 2.1: A0 = Q0 Lambda0 Q0^-1) and the small dense host
// factorisations call the standard Fortran LAPACK symbols found in the
// process (a Python process that imported torch has them in libtorch_cpu),
// or in the shared library named by LYAP_LAPACK_LIB.
#include "lapack_host.h"

#include <dlfcn.h>

#include <cstdlib>
#include <mutex>

namespace lyap {

namespace {
std::once_flag g_once;
LapackFns g_fns;

void* find(void* lib, const char* name) {
  void* p = dlsym(RTLD_DEFAULT, name);
  if (!p && lib) p = dlsym(lib, name);
  return p;
}

void resolve() {
  void* lib = nullptr;
  if (const char* env = std::getenv("LYAP_LAPACK_LIB")) lib = dlopen(env, RTLD_NOW | RTLD_LOCAL);
  if (!dlsym(RTLD_DEFAULT, "dgeev_") && !lib) {
    const char* cands[] = {"liblapack.so.3", "liblapack.so", "libopenblas.so.0", "libtorch_cpu.so"};
    for (const char* c : cands) {
      lib = dlopen(c, RTLD_NOW | RTLD_LOCAL);
      if (lib && dlsym(lib, "dgeev_")) break;
      lib = nullptr;
    }
  }
  g_fns.dgeev = reinterpret_cast<LapackFns::dgeev_t>(find(lib, "dgeev_"));
  g_fns.dgetrf = reinterpret_cast<LapackFns::dgetrf_t>(find(lib, "dgetrf_"));
  g_fns.dgetrs = reinterpret_cast<LapackFns::dgetrs_t>(find(lib, "dgetrs_"));
  g_fns.dgesdd = reinterpret_cast<LapackFns::dgesdd_t>(find(lib, "dgesdd_"));
  g_fns.dgeqrf = reinterpret_cast<LapackFns::dgeqrf_t>(find(lib, "dgeqrf_"));
  g_fns.dorgqr = reinterpret_cast<LapackFns::dorgqr_t>(find(lib, "dorgqr_"));
}
}  // namespace

const LapackFns& lapack() {
  std::call_once(g_once, resolve);
  return g_fns;
}

}  // namespace lyap
