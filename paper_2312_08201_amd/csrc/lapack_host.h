// Run-time resolved host LAPACK entry points (Fortran ABI, 32-bit integers).
#pragma once

namespace lyap {

struct LapackFns {
  typedef void (*dgeev_t)(const char*, const char*, const int*, double*, const int*, double*,
                          double*, double*, const int*, double*, const int*, double*, const int*,
                          int*);
  typedef void (*dgetrf_t)(const int*, const int*, double*, const int*, int*, int*);
  typedef void (*dgetrs_t)(const char*, const int*, const int*, const double*, const int*,
                           const int*, double*, const int*, int*);
  typedef void (*dgesdd_t)(const char*, const int*, const int*, double*, const int*, double*,
                           double*, const int*, double*, const int*, double*, const int*, int*,
                           int*);
  typedef void (*dgeqrf_t)(const int*, const int*, double*, const int*, double*, double*,
                           const int*, int*);
  typedef void (*dorgqr_t)(const int*, const int*, const int*, double*, const int*,
                           const double*, double*, const int*, int*);
  dgeev_t dgeev = nullptr;
  dgetrf_t dgetrf = nullptr;
  dgetrs_t dgetrs = nullptr;
  dgesdd_t dgesdd = nullptr;
  dgeqrf_t dgeqrf = nullptr;
  dorgqr_t dorgqr = nullptr;
};

const LapackFns& lapack();

}  // namespace lyap
