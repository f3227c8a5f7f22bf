// Stability filter for parameter sweeps: the number of eigenvalues of
//     A(d) = A0 - U diag(d) V^T
// in the open right half-plane, for many d at once, from the seed alone.
//
// The multi-agent importance example of Section 4 discards every parameter
// sample whose A(d) has an eigenvalue with a non-negative real part.  Here
// that decision uses the low-rank structure instead of a dense eigensolve
// per sample.  With G(s) = V^T (s I - A0)^-1 U (r x r),
//     det(s I - A(d)) = det(s I - A0) det(I + D G(s)),
// and A0 is stable, so the eigenvalues of A(d) in the right half-plane are
// the zeros there of f(s) = det(I + D G(s)), which is analytic there and
// tends to 1 at infinity.  By the argument principle on the imaginary axis
// and the conjugate symmetry f(-i w) = conj f(i w), their number is
//     Z = -(1/pi) * (change of arg f(i w) for w from 0 to infinity).
// In the seed's eigenbasis G(i w) = sum_mu Vh_mu Uh_mu^T / (i w - mu), an
// O(r^2 n) sum per frequency that every sample shares.  The phase is
// followed on a frequency grid dense around every eigenvalue of A0 (steps of
// |Re mu| / 4 within 4 |Re mu| of Im mu), uniform at 1/2048 of the spectral
// radius over [0, 2 rho], and geometric out to 1000 (rho + 1), or further for
// large |d| (until ||D G|| is small enough that f cannot wind).  A phase step
// above pi/2 means an eigenvalue of A(d) close to the axis; the samples with
// such a step get a second pass that splits each of those steps into 16
// sub-steps with f evaluated directly from the eigen expansion, and splits
// again where a sub-step still exceeds pi/2 (four levels, 16^4 times finer).
// A sample stays flagged when that does not resolve it, when |f - 1| >= 1/2
// at the last frequency, or when the total is not within 1/4 of an integer
// multiple of pi.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace lyap {
namespace {

constexpr int kStabChunk = 512;  // frequencies per thread of the phase kernel
constexpr int kStabMaxR = 8;

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// G[l][a][b] (complex, interleaved) = sum over the eigenvalues mu of A0 of
// Vh[a][mu] Uh[b][mu] / (i omega_l - mu); one wavefront per (l, a b).
__global__ void __launch_bounds__(64) k_stab_G(const double* __restrict__ lam,
                                               const double* __restrict__ Uh,
                                               const double* __restrict__ Vh, int n, int h, int ld,
                                               int r, const double* __restrict__ omega,
                                               double* __restrict__ G) {
  const int l = blockIdx.x, ab = blockIdx.y, a = ab / r, b = ab % r;
  const double w = omega[l];
  const int units = h + (n - 2 * h);
  double sr = 0.0, si = 0.0;
  for (int u = threadIdx.x; u < units; u += 64) {
    if (u < h) {
      // pair: lambda = al + i be (be > 0) and its conjugate, coefficients z and conj(z)
      const int q = 2 * u;
      const double al = lam[q], be = lam[ld + q];
      const double vr = Vh[(long)a * ld + q], vi = Vh[(long)a * ld + q + 1];
      const double ur = Uh[(long)b * ld + q], ui = Uh[(long)b * ld + q + 1];
      const double zr = vr * ur - vi * ui, zi = vr * ui + vi * ur;
      const double d1i = w - be, n1 = al * al + d1i * d1i;
      const double d2i = w + be, n2 = al * al + d2i * d2i;
      sr += (-zr * al + zi * d1i) / n1 + (-zr * al - zi * d2i) / n2;
      si += (-zi * al - zr * d1i) / n1 + (zi * al - zr * d2i) / n2;
    } else {
      const int q = 2 * h + (u - h);
      const double al = lam[q];
      const double z = Vh[(long)a * ld + q] * Uh[(long)b * ld + q];
      const double nn = al * al + w * w;
      sr += -z * al / nn;
      si += -z * w / nn;
    }
  }
  sr = wsum(sr);
  si = wsum(si);
  if (threadIdx.x == 0) {
    G[((long)l * r * r + ab) * 2] = sr;
    G[((long)l * r * r + ab) * 2 + 1] = si;
  }
}

// det(I + D G_l) by Gaussian elimination with partial pivoting (compile-time
// indices throughout, so the matrix stays in registers)
template <int R>
__device__ inline void det_l(const double* __restrict__ Gl, const double (&dp)[R], double& fr,
                             double& fi) {
  double Mr[R * R], Mi[R * R];
#pragma unroll
  for (int a = 0; a < R; ++a)
#pragma unroll
    for (int b = 0; b < R; ++b) {
      Mr[a * R + b] = (a == b ? 1.0 : 0.0) + dp[a] * Gl[(a * R + b) * 2];
      Mi[a * R + b] = dp[a] * Gl[(a * R + b) * 2 + 1];
    }
  double dr = 1.0, di = 0.0;
#pragma unroll
  for (int c = 0; c < R; ++c) {
#pragma unroll
    for (int i = c + 1; i < R; ++i) {
      const bool sw = Mr[i * R + c] * Mr[i * R + c] + Mi[i * R + c] * Mi[i * R + c] >
                      Mr[c * R + c] * Mr[c * R + c] + Mi[c * R + c] * Mi[c * R + c];
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const double xr = Mr[c * R + k], yr = Mr[i * R + k];
        const double xi = Mi[c * R + k], yi = Mi[i * R + k];
        Mr[c * R + k] = sw ? yr : xr;
        Mr[i * R + k] = sw ? xr : yr;
        Mi[c * R + k] = sw ? yi : xi;
        Mi[i * R + k] = sw ? xi : yi;
      }
      dr = sw ? -dr : dr;
      di = sw ? -di : di;
    }
    const double pr = Mr[c * R + c], pi = Mi[c * R + c];
    const double tr = dr * pr - di * pi, ti = dr * pi + di * pr;
    dr = tr;
    di = ti;
    const double pn = pr * pr + pi * pi;
    const double ir = pn > 0.0 ? pr / pn : 0.0, ii = pn > 0.0 ? -pi / pn : 0.0;
#pragma unroll
    for (int i = c + 1; i < R; ++i) {
      const double fr_ = Mr[i * R + c] * ir - Mi[i * R + c] * ii;
      const double fi_ = Mr[i * R + c] * ii + Mi[i * R + c] * ir;
#pragma unroll
      for (int k = c + 1; k < R; ++k) {
        Mr[i * R + k] -= fr_ * Mr[c * R + k] - fi_ * Mi[c * R + k];
        Mi[i * R + k] -= fr_ * Mi[c * R + k] + fi_ * Mr[c * R + k];
      }
    }
  }
  fr = dr;
  fi = di;
}

// Thread t: sample p = t % P, frequency chunk c = t / P.  Sums the phase
// steps arg(f_l / f_(l-1)) for l = c kStabChunk + 1, ..., (c + 1) kStabChunk
// (below L); the last chunk adds the step from the last frequency to f = 1
// at infinity.
template <int R>
__global__ void __launch_bounds__(256) k_stab_phase(const double* __restrict__ G, int L,
                                                    const double* __restrict__ d, long P,
                                                    int nchunk, double* __restrict__ part,
                                                    int* __restrict__ pflag) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P * nchunk) return;
  const long p = t % P;
  const int c = (int)(t / P);
  double dp[R];
#pragma unroll
  for (int a = 0; a < R; ++a) dp[a] = d[p * R + a];
  const int lstart = c * kStabChunk;
  const int l1 = min(L, lstart + 1 + kStabChunk);
  double pr, pim;
  det_l<R>(G + (long)lstart * R * R * 2, dp, pr, pim);
  double sum = 0.0;
  int flag = (pr == 0.0 && pim == 0.0) ? 8 : 0;
  for (int l = lstart + 1; l < l1; ++l) {
    double fr, fi;
    det_l<R>(G + (long)l * R * R * 2, dp, fr, fi);
    // arg(f conj(fprev))
    const double step = atan2(fi * pr - fr * pim, fr * pr + fi * pim);
    if (fabs(step) > 0.5 * M_PI) flag |= 1;
    if (fr == 0.0 && fi == 0.0) flag |= 8;
    sum += step;
    pr = fr;
    pim = fi;
  }
  if (c == nchunk - 1) {
    const double er = pr - 1.0;
    if (er * er + pim * pim >= 0.25) flag |= 2;
    sum += -atan2(pim, pr);  // from f_last to 1
  }
  part[t] = sum;
  pflag[t] = flag;
}

// f(i w) = det(I + D G(i w)) with G evaluated directly from the eigen expansion
// (the same sum as k_stab_G, one thread)
template <int R>
__device__ inline void f_direct(const double* __restrict__ lam, const double* __restrict__ Uh,
                                const double* __restrict__ Vh, int n, int h, int ld, double w,
                                const double (&dp)[R], double& fr, double& fi) {
  double G[R * R * 2];
#pragma unroll
  for (int e = 0; e < R * R * 2; ++e) G[e] = 0.0;
  const int units = h + (n - 2 * h);
  for (int u = 0; u < units; ++u) {
    if (u < h) {
      const int q = 2 * u;
      const double al = lam[q], be = lam[ld + q];
      const double d1i = w - be, n1 = al * al + d1i * d1i;
      const double d2i = w + be, n2 = al * al + d2i * d2i;
#pragma unroll
      for (int a = 0; a < R; ++a) {
        const double vr = Vh[(long)a * ld + q], vi = Vh[(long)a * ld + q + 1];
#pragma unroll
        for (int b = 0; b < R; ++b) {
          const double ur = Uh[(long)b * ld + q], ui = Uh[(long)b * ld + q + 1];
          const double zr = vr * ur - vi * ui, zi = vr * ui + vi * ur;
          G[(a * R + b) * 2] += (-zr * al + zi * d1i) / n1 + (-zr * al - zi * d2i) / n2;
          G[(a * R + b) * 2 + 1] += (-zi * al - zr * d1i) / n1 + (zi * al - zr * d2i) / n2;
        }
      }
    } else {
      const int q = 2 * h + (u - h);
      const double al = lam[q];
      const double nn = al * al + w * w;
#pragma unroll
      for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = 0; b < R; ++b) {
          const double z = Vh[(long)a * ld + q] * Uh[(long)b * ld + q];
          G[(a * R + b) * 2] += -z * al / nn;
          G[(a * R + b) * 2 + 1] += -z * w / nn;
        }
    }
  }
  det_l<R>(G, dp, fr, fi);
}

struct StabSeed {
  const double* lam;
  const double* Uh;
  const double* Vh;
  int n, h, ld;
};

constexpr int kRefineSplit = 16;  // sub-intervals per refinement level

// Phase change of f over [wa, wb] (f known at both ends), from kRefineSplit
// direct evaluations; a sub-step above pi/2 is split again, DEPTH more times.
// bad is set when a sub-step at the last level still exceeds pi/2.
template <int DEPTH, int R>
__device__ double phase_refined(const StabSeed& S, const double (&dp)[R], double wa, double wb,
                                double far, double fai, double fbr, double fbi, int& bad) {
  double sum = 0.0, pr = far, pim = fai, wp = wa;
  for (int k = 1; k <= kRefineSplit; ++k) {
    const double w = k == kRefineSplit ? wb : wa + (wb - wa) * k / kRefineSplit;
    double fr, fi;
    if (k == kRefineSplit) {
      fr = fbr;
      fi = fbi;
    } else {
      f_direct<R>(S.lam, S.Uh, S.Vh, S.n, S.h, S.ld, w, dp, fr, fi);
    }
    double step = atan2(fi * pr - fr * pim, fr * pr + fi * pim);
    if (fabs(step) > 0.5 * M_PI) {
      if constexpr (DEPTH > 0) step = phase_refined<DEPTH - 1, R>(S, dp, wp, w, pr, pim, fr, fi, bad);
      else bad = 1;
    }
    sum += step;
    pr = fr;
    pim = fi;
    wp = w;
  }
  return sum;
}

// Second pass for the samples idx[0..m-1] that the grid flagged: the whole
// phase walk again, each step above pi/2 refined by direct evaluations.
// Writes count and flag of those samples (flag keeps bits 2, 8 of the walk).
template <int R>
__global__ void __launch_bounds__(64) k_stab_refine(StabSeed S, const double* __restrict__ G,
                                                    const double* __restrict__ omega, int L,
                                                    const double* __restrict__ d,
                                                    const int* __restrict__ idx, int m,
                                                    int* __restrict__ count, int* __restrict__ flag) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m) return;
  const long p = idx[t];
  double dp[R];
#pragma unroll
  for (int a = 0; a < R; ++a) dp[a] = d[p * R + a];
  double pr, pim;
  det_l<R>(G, dp, pr, pim);
  int bad = 0, f = (pr == 0.0 && pim == 0.0) ? 8 : 0;
  double sum = 0.0;
  for (int l = 1; l < L; ++l) {
    double fr, fi;
    det_l<R>(G + (long)l * R * R * 2, dp, fr, fi);
    double step = atan2(fi * pr - fr * pim, fr * pr + fi * pim);
    if (fabs(step) > 0.5 * M_PI)
      step = phase_refined<3, R>(S, dp, omega[l - 1], omega[l], pr, pim, fr, fi, bad);
    if (fr == 0.0 && fi == 0.0) f |= 8;
    sum += step;
    pr = fr;
    pim = fi;
  }
  {
    const double er = pr - 1.0;
    if (er * er + pim * pim >= 0.25) f |= 2;
    sum += -atan2(pim, pr);
  }
  if (bad) f |= 1;
  const double z = -sum / M_PI;
  const double zr = rint(z);
  // a non-finite total (NaN or Inf along the walk) fails the comparison and is flagged
  if (!(fabs(z - zr) <= 0.25) || zr < 0.0) f |= 4;
  count[p] = (zr >= 0.0 && zr < 2147483647.0) ? (int)zr : 0;
  flag[p] = f;
}

__global__ void k_stab_reduce(const double* __restrict__ part, const int* __restrict__ pflag,
                              long P, int nchunk, int* __restrict__ count, int* __restrict__ flag) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double sum = 0.0;
  int f = 0;
  for (int c = 0; c < nchunk; ++c) {
    sum += part[(long)c * P + p];
    f |= pflag[(long)c * P + p];
  }
  const double z = -sum / M_PI;
  const double zr = rint(z);
  // a non-finite total (NaN or Inf along the walk) fails the comparison and is flagged
  if (!(fabs(z - zr) <= 0.25) || zr < 0.0) f |= 4;
  count[p] = (zr >= 0.0 && zr < 2147483647.0) ? (int)zr : 0;
  flag[p] = f;
}

// Frequencies (ascending, from 0) for the seed's spectrum; the geometric tail
// reaches at least `reach`.
std::vector<double> stability_grid(const std::vector<double>& lam_h, int n, int h, long ld,
                                   double reach) {
  std::vector<double> w{0.0};
  double amin = INFINITY, rho = 0.0;
  const int units = h + (n - 2 * h);
  for (int u = 0; u < units; ++u) {
    const int q = u < h ? 2 * u : 2 * h + (u - h);
    const double al = std::fabs(lam_h[q]), be = std::fabs(lam_h[ld + q]);
    amin = std::min(amin, al);
    rho = std::max(rho, std::hypot(al, be));
    for (int j = -16; j <= 16; ++j) {
      const double x = be + j * 0.25 * al;
      if (x > 0.0) w.push_back(x);
    }
  }
  for (int j = 1; j <= 4096; ++j) w.push_back(2.0 * rho * j / 4096.0);
  const double top = std::max(1000.0 * (rho + 1.0), reach);
  for (double x = std::max(amin / 64.0, 1e-300); x < top; x *= 1.02) w.push_back(x);
  w.push_back(top);
  std::sort(w.begin(), w.end());
  w.erase(std::unique(w.begin(), w.end()), w.end());
  return w;
}

template <int R>
void launch_phase(const double* G, int L, const double* d, long P, int nchunk, double* part,
                  int* pflag, hipStream_t st) {
  const long threads = P * nchunk;
  hipLaunchKernelGGL(k_stab_phase<R>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, G,
                     L, d, P, nchunk, part, pflag);
}

void unstable_impl(lyap_seed_s* sd, int64_t P, const double* d, int* count, int* flag,
                   hipStream_t st) {
  LYAP_REQUIRE(P >= 0 && P < (1LL << 31), LYAP_E_INVAL, "P out of [0, 2^31)");
  if (P == 0) return;
  LYAP_REQUIRE(d && count && flag, LYAP_E_INVAL, "null pointer");
  LYAP_REQUIRE(sd->basis == LYAP_BASIS_EIG, LYAP_E_UNSUPPORTED,
               "the stability filter needs the seed's eigenbasis");
  LYAP_REQUIRE(!sd->projected, LYAP_E_UNSUPPORTED, "a projected seed has no stable A0");
  LYAP_REQUIRE(sd->r <= kStabMaxR, LYAP_E_UNSUPPORTED, "stability filter limited to r <= 8");
  const long ld = sd->ld;
  const int n = (int)sd->n, h = (int)sd->h, r = (int)sd->r;
  std::vector<double> lam_h(2 * ld);
  LYAP_HIP(hipMemcpyAsync(lam_h.data(), sd->lam.p, 2 * ld * sizeof(double), hipMemcpyDeviceToHost,
                          st));
  LYAP_HIP(hipStreamSynchronize(st));
  // Beyond w, ||D G(i w)|| <= max|d| sum_mu ||Vh_mu|| ||Uh_mu|| / (w - rho); the tail
  // reaches the w where that is 0.04, so |det(I + D G) - 1| < 1/2 for r <= 8.
  double reach = 0.0;
  {
    std::vector<double> dh((size_t)P * r), uh((size_t)r * ld), vh((size_t)r * ld);
    LYAP_HIP(hipMemcpyAsync(dh.data(), d, dh.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    LYAP_HIP(hipMemcpyAsync(uh.data(), sd->Uh.p, uh.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    LYAP_HIP(hipMemcpyAsync(vh.data(), sd->Vh.p, vh.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    LYAP_HIP(hipStreamSynchronize(st));
    double dmax = 0.0, wsum = 0.0, rho = 0.0;
    for (double x : dh) {
      LYAP_REQUIRE(std::isfinite(x), LYAP_E_INVAL, "d has a non-finite entry");
      dmax = std::max(dmax, std::fabs(x));
    }
    const int units = h + (n - 2 * h);
    for (int u = 0; u < units; ++u) {
      const bool pair = u < h;
      const int q = pair ? 2 * u : 2 * h + (u - h);
      double nu = 0.0, nv = 0.0;
      for (int a = 0; a < r; ++a) {
        nu += uh[(size_t)a * ld + q] * uh[(size_t)a * ld + q];
        nv += vh[(size_t)a * ld + q] * vh[(size_t)a * ld + q];
        if (pair) {
          nu += uh[(size_t)a * ld + q + 1] * uh[(size_t)a * ld + q + 1];
          nv += vh[(size_t)a * ld + q + 1] * vh[(size_t)a * ld + q + 1];
        }
      }
      wsum += (pair ? 2.0 : 1.0) * std::sqrt(nu * nv);
      rho = std::max(rho, std::hypot(lam_h[q], lam_h[ld + q]));
    }
    reach = rho + 25.0 * dmax * wsum;
  }
  const std::vector<double> w = stability_grid(lam_h, n, h, ld, reach);
  const int L = (int)w.size();
  const int nchunk = (L - 1 + kStabChunk - 1) / kStabChunk;
  DevBuf wd(w.size() * sizeof(double)), G((size_t)L * r * r * 2 * sizeof(double)),
      part((size_t)P * nchunk * sizeof(double)), pflag((size_t)P * nchunk * sizeof(int));
  LYAP_HIP(hipMemcpyAsync(wd.p, w.data(), wd.bytes, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_stab_G, dim3((unsigned)L, (unsigned)(r * r)), dim3(64), 0, st,
                     sd->lam.as<double>(), sd->Uh.as<double>(), sd->Vh.as<double>(), n, h, (int)ld,
                     r, wd.as<double>(), G.as<double>());
  LYAP_HIP(hipGetLastError());
  switch (r) {
    case 1: launch_phase<1>(G.as<double>(), L, d, P, nchunk, part.as<double>(), pflag.as<int>(), st); break;
    case 2: launch_phase<2>(G.as<double>(), L, d, P, nchunk, part.as<double>(), pflag.as<int>(), st); break;
    case 3: launch_phase<3>(G.as<double>(), L, d, P, nchunk, part.as<double>(), pflag.as<int>(), st); break;
    case 4: launch_phase<4>(G.as<double>(), L, d, P, nchunk, part.as<double>(), pflag.as<int>(), st); break;
    case 5: launch_phase<5>(G.as<double>(), L, d, P, nchunk, part.as<double>(), pflag.as<int>(), st); break;
    case 6: launch_phase<6>(G.as<double>(), L, d, P, nchunk, part.as<double>(), pflag.as<int>(), st); break;
    case 7: launch_phase<7>(G.as<double>(), L, d, P, nchunk, part.as<double>(), pflag.as<int>(), st); break;
    default: launch_phase<8>(G.as<double>(), L, d, P, nchunk, part.as<double>(), pflag.as<int>(), st); break;
  }
  LYAP_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_stab_reduce, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st,
                     part.as<double>(), pflag.as<int>(), (long)P, nchunk, count, flag);
  LYAP_HIP(hipGetLastError());
  // second pass over the flagged samples: steps above pi/2 refined by direct evaluations
  std::vector<int> fl(P);
  LYAP_HIP(hipMemcpyAsync(fl.data(), flag, P * sizeof(int), hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipStreamSynchronize(st));
  std::vector<int> idx;
  for (int64_t p = 0; p < P; ++p)
    if (fl[p] & 1) idx.push_back((int)p);
  if (!idx.empty()) {
    const int m = (int)idx.size();
    DevBuf idd(idx.size() * sizeof(int));
    LYAP_HIP(hipMemcpyAsync(idd.p, idx.data(), idd.bytes, hipMemcpyHostToDevice, st));
    StabSeed S{sd->lam.as<double>(), sd->Uh.as<double>(), sd->Vh.as<double>(), n, h, (int)ld};
    const dim3 grid((unsigned)((m + 63) / 64)), block(64);
    const double* Gp = G.as<double>();
    const double* wp = wd.as<double>();
    const int* ip = idd.as<int>();
    switch (r) {
      case 1: hipLaunchKernelGGL(k_stab_refine<1>, grid, block, 0, st, S, Gp, wp, L, d, ip, m, count, flag); break;
      case 2: hipLaunchKernelGGL(k_stab_refine<2>, grid, block, 0, st, S, Gp, wp, L, d, ip, m, count, flag); break;
      case 3: hipLaunchKernelGGL(k_stab_refine<3>, grid, block, 0, st, S, Gp, wp, L, d, ip, m, count, flag); break;
      case 4: hipLaunchKernelGGL(k_stab_refine<4>, grid, block, 0, st, S, Gp, wp, L, d, ip, m, count, flag); break;
      case 5: hipLaunchKernelGGL(k_stab_refine<5>, grid, block, 0, st, S, Gp, wp, L, d, ip, m, count, flag); break;
      case 6: hipLaunchKernelGGL(k_stab_refine<6>, grid, block, 0, st, S, Gp, wp, L, d, ip, m, count, flag); break;
      case 7: hipLaunchKernelGGL(k_stab_refine<7>, grid, block, 0, st, S, Gp, wp, L, d, ip, m, count, flag); break;
      default: hipLaunchKernelGGL(k_stab_refine<8>, grid, block, 0, st, S, Gp, wp, L, d, ip, m, count, flag); break;
    }
    LYAP_HIP(hipGetLastError());
    LYAP_HIP(hipStreamSynchronize(st));
  }
  LYAP_HIP(hipStreamSynchronize(st));  // the work buffers are freed on return
}

}  // namespace
}  // namespace lyap

using namespace lyap;

extern "C" {

lyap_status seed_unstable_count(lyap_seed sd, int64_t P, const double* d_dev, int32_t* count_dev,
                                int32_t* flag_dev, void* hip_stream) {
  if (!sd) return LYAP_E_INVAL;
  LYAP_TRY(unstable_impl(sd, P, d_dev, count_dev, flag_dev, (hipStream_t)hip_stream));
  return LYAP_OK;
}

}  // extern "C"
