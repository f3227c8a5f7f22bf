// Host-only driver for the library's real Schur decomposition (schur_host.cpp),
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitizers.py.  For each case it checks A = Z T Z^T,
// Z^T Z = I and the quasi-triangular shape of T, and prints one line.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2312_08201_amd/csrc/schur_host.h"

static unsigned long long state = 88172645463325252ULL;
static double urand() {  // xorshift64, uniform in [-1, 1)
  state ^= state << 13;
  state ^= state >> 7;
  state ^= state << 17;
  return (double)(state >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}

static int check(int n, const std::vector<double>& A, const char* name) {
  std::vector<double> T((size_t)n * n), Z((size_t)n * n);
  int it = 0;
  if (!lyap::real_schur(n, A.data(), T.data(), Z.data(), &it)) {
    std::printf("%s n=%d: no convergence\n", name, n);
    return 1;
  }
  double na = 0, rec = 0, orth = 0, low = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double zt = 0, zz = 0;
      for (int k = 0; k < n; ++k) {
        double tz = 0;
        for (int l = 0; l < n; ++l) tz += T[(size_t)k * n + l] * Z[(size_t)j * n + l];
        zt += Z[(size_t)i * n + k] * tz;
        zz += Z[(size_t)k * n + i] * Z[(size_t)k * n + j];
      }
      const double a = A[(size_t)i * n + j];
      na += a * a;
      rec += (zt - a) * (zt - a);
      orth += (zz - (i == j)) * (zz - (i == j));
      if (i > j + 1) low += std::fabs(T[(size_t)i * n + j]);
    }
  const double r = std::sqrt(rec / (na > 0 ? na : 1.0)), o = std::sqrt(orth);
  const bool ok = r <= 1e-12 && o <= 1e-12 * n && low == 0.0;
  std::printf("%s n=%d: reconstruction %.2e, orthogonality %.2e, below subdiagonal %.1e: %s\n",
              name, n, r, o, low, ok ? "ok" : "FAIL");
  return ok ? 0 : 1;
}

int main() {
  int bad = 0;
  const int sizes[] = {1, 2, 3, 5, 8, 17, 40, 96};
  for (int n : sizes) {
    std::vector<double> A((size_t)n * n);
    for (auto& v : A) v = urand();
    bad += check(n, A, "random");
    // rotation blocks: complex pairs with equal real parts
    std::vector<double> R((size_t)n * n, 0.0);
    for (int k = 0; k + 1 < n; k += 2) {
      R[(size_t)k * n + k] = R[(size_t)(k + 1) * n + k + 1] = -0.5;
      R[(size_t)k * n + k + 1] = 1.0 + k;
      R[(size_t)(k + 1) * n + k] = -1.0 - k;
    }
    if (n % 2) R[(size_t)(n - 1) * n + n - 1] = -2.0;
    bad += check(n, R, "rotations");
    // a Jordan-like (defective) upper bidiagonal block
    std::vector<double> J((size_t)n * n, 0.0);
    for (int k = 0; k < n; ++k) {
      J[(size_t)k * n + k] = -1.0;
      if (k + 1 < n) J[(size_t)k * n + k + 1] = 1.0;
    }
    bad += check(n, J, "jordan");
  }
  std::printf(bad ? "FAILED %d\n" : "ALL OK\n", bad);
  return bad ? 1 : 0;
}
