// Shifted-family solve for one-column parameters (r = 1).
//
// With r = 1 the capacitance system of a parameter d is (I - d K) y = d c0
// (K the capacitance operator, c0 = V^T X0).  For d != 0 it is the shifted
// system (sigma I - K) y = c0 with sigma = 1/d, and Krylov spaces are
// invariant under shifts: one Arnoldi process K V_j = V_(j+1) Hb_j started
// from c0 serves every sigma, and GMRES for the shift sigma minimises
// || beta e1 - (sigma I_bar - Hb_j) z || (I_bar = [I; 0]).  Each Arnoldi step
// is one seed apply (the same kernels as lyap_seed_apply) and a CGS2
// orthogonalisation; each shift keeps its own Givens rotations and rotated
// right-hand side, one thread per shift.  The cost grows with the number of
// Arnoldi steps the hardest shift needs, almost not with the number of
// shifts.  No preconditioner: the block-diagonal preconditioner of eq:prec
// depends on d and would break the shift invariance.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace lyap {
namespace {

constexpr int NT = 256;
constexpr int kMaxSteps = 2048;
constexpr int kPollEvery = 4;  // Arnoldi steps between convergence checks on the host

__device__ inline double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// h[j] = ||w||, v_j = w / h[j]   (one workgroup)
__global__ void __launch_bounds__(NT) k_sh_normalize(const double* __restrict__ w, int n,
                                                     double* __restrict__ hj,
                                                     double* __restrict__ vout) {
  __shared__ double red[NT];
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += NT) acc += w[k] * w[k];
  const double nrm = sqrt(block_sum(acc, red));
  if (threadIdx.x == 0) hj[0] = nrm;
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int k = threadIdx.x; k < n; k += NT) vout[k] = w[k] * inv;
}

// One Givens step of every unconverged shift for Arnoldi column j (rows 0..j+1
// of Hb in Hcol).  conv[p] >= 0: converged with conv[p] columns (or d = 0).
__global__ void k_sh_shift(const double* __restrict__ Hcol, int j, const double* __restrict__ sig,
                           int P, int mmax, double* __restrict__ cs, double* __restrict__ sn,
                           double* __restrict__ g, double* __restrict__ resid,
                           int* __restrict__ conv, double tol_abs, int* __restrict__ unconv,
                           int last) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P || conv[p] >= 0) return;
  const double sigma = sig[p];
  // per-shift arrays are stored element-major ([i * P + p]): coalesced over shifts
  const long Pl = P;
  // column j of (sigma I_bar - Hb): -h_ij, plus sigma on row j
  double t = -Hcol[0] + (j == 0 ? sigma : 0.0);
  for (int i = 0; i < j; ++i) {
    const double nx = -Hcol[i + 1] + (i + 1 == j ? sigma : 0.0);
    // row i+1 after rotation i (row i's final value is not kept)
    t = -sn[i * Pl + p] * t + cs[i * Pl + p] * nx;
  }
  const double hs = -Hcol[j + 1];
  const double rho = hypot(t, hs);
  const double cj = rho > 0.0 ? t / rho : 1.0, sj = rho > 0.0 ? hs / rho : 0.0;
  cs[j * Pl + p] = cj;
  sn[j * Pl + p] = sj;
  const double gj = g[j * Pl + p];
  g[j * Pl + p] = cj * gj;
  g[(j + 1) * Pl + p] = -sj * gj;
  const double r = fabs(g[(j + 1) * Pl + p]);
  resid[p] = r;
  if (r <= tol_abs || last) conv[p] = j + 1;
  else atomicAdd(unconv, 1);
}

// z (ncol entries) solving R z = g, R the rotated (sigma I_bar - Hb) restricted
// to its first ncol columns; columns of R are rebuilt one at a time (back to
// front) from Hb and the shift's rotations.  x and col: per-shift scratch.
__global__ void k_sh_solve(const double* __restrict__ Hb, int ldh, const double* __restrict__ sig,
                           int P, int mmax, const double* __restrict__ cs,
                           const double* __restrict__ sn, const double* __restrict__ g,
                           const int* __restrict__ conv, double* __restrict__ x,
                           double* __restrict__ col, double* __restrict__ Z, int ldz) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int nc = conv[p];
  double* zp = Z + (long)p * ldz;
  for (int i = 0; i < ldz; ++i) zp[i] = 0.0;
  if (nc <= 0) return;
  const double sigma = sig[p];
  const long Pl = P;
  for (int i = 0; i < nc; ++i) x[i * Pl + p] = g[i * Pl + p];
  for (int cc = nc - 1; cc >= 0; --cc) {
    const double* h = Hb + (long)cc * ldh;
    for (int i = 0; i <= cc + 1; ++i) col[i * Pl + p] = -h[i] + (i == cc ? sigma : 0.0);
    for (int i = 0; i <= cc; ++i) {  // rotations 0..cc on rows (i, i+1)
      const double a = col[i * Pl + p], b = col[(i + 1) * Pl + p];
      const double ci = cs[i * Pl + p], si = sn[i * Pl + p];
      col[i * Pl + p] = ci * a + si * b;
      col[(i + 1) * Pl + p] = -si * a + ci * b;
    }
    const double zc = x[cc * Pl + p] / col[cc * Pl + p];
    zp[cc] = zc;
    for (int i = 0; i < cc; ++i) x[i * Pl + p] -= zc * col[i * Pl + p];
  }
}

// CGS2 of w against v_0 .. v_j and the new basis vector, in one workgroup:
// each wavefront takes every 16th dot product (wavefront reduction), the
// update runs over the elements.  h: column j of Hb (rows 0..j+1).
constexpr int OT = 1024;
__global__ void __launch_bounds__(OT) k_sh_orth(const double* __restrict__ V, long ld,
                                                double* __restrict__ w, int n, int j,
                                                double* __restrict__ h, double* __restrict__ vout) {
  __shared__ double hc[kMaxSteps + 1];
  __shared__ double red[OT / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = threadIdx.x; i <= j; i += OT) h[i] = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    __syncthreads();
    for (int i = wave; i <= j; i += OT / 64) {
      const double* v = V + (long)i * ld;
      double acc = 0.0;
      for (int k = lane; k < n; k += 64) acc += v[k] * w[k];
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
      if (lane == 0) hc[i] = acc;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += OT) {
      double acc = w[k];
      for (int i = 0; i <= j; ++i) acc -= hc[i] * V[(long)i * ld + k];
      w[k] = acc;
    }
    for (int i = threadIdx.x; i <= j; i += OT) h[i] += hc[i];
  }
  __syncthreads();
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += OT) acc += w[k] * w[k];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) red[wave] = acc;
  __syncthreads();
  double nrm = 0.0;
  for (int q = 0; q < OT / 64; ++q) nrm += red[q];
  nrm = sqrt(nrm);
  if (threadIdx.x == 0) h[j + 1] = nrm;
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int k = threadIdx.x; k < n; k += OT) vout[k] = w[k] * inv;
}

void shifted_impl(lyap_seed_s* sd, int64_t P, const double* d_host, const lyap_solve_opts* in,
                  double* Y_dev, lyap_result* res, hipStream_t st) {
  LYAP_REQUIRE(sd->r == 1, LYAP_E_UNSUPPORTED, "the shifted-family solve needs r = 1");
  LYAP_REQUIRE(!sd->projected, LYAP_E_UNSUPPORTED, "projected seeds are solved by ek_sweep");
  LYAP_REQUIRE(P >= 1 && d_host && res, LYAP_E_INVAL, "bad argument");
  const double tol = in && in->tol > 0 ? in->tol : 1e-12;
  const int mmax = std::min(kMaxSteps, in && in->max_iter > 0 ? (int)in->max_iter : 600);
  const long n = sd->n, ld = sd->ld;
  std::vector<double> sig_h(P);
  std::vector<int> conv_h(P);
  for (int64_t p = 0; p < P; ++p) {
    LYAP_REQUIRE(std::isfinite(d_host[p]), LYAP_E_INVAL, "non-finite parameter");
    conv_h[p] = d_host[p] == 0.0 ? 0 : -1;
    sig_h[p] = d_host[p] == 0.0 ? 0.0 : 1.0 / d_host[p];
  }
  const long mpad = pad_to(mmax + 1, 128);
  DevBuf V((size_t)mpad * ld * sizeof(double)), w(ld * sizeof(double)),
      Hb((size_t)(mmax + 2) * mmax * sizeof(double)), sig(P * sizeof(double)),
      cs((size_t)P * mmax * sizeof(double)), sn((size_t)P * mmax * sizeof(double)),
      g((size_t)P * (mmax + 1) * sizeof(double)), resid(P * sizeof(double)),
      conv(P * sizeof(int)), unconv(sizeof(int)), c0p(ld * sizeof(double));
  const int ldh = mmax + 2;
  LYAP_HIP(hipMemsetAsync(V.p, 0, V.bytes, st));
  LYAP_HIP(hipMemsetAsync(w.p, 0, w.bytes, st));
  LYAP_HIP(hipMemsetAsync(Hb.p, 0, Hb.bytes, st));
  LYAP_HIP(hipMemsetAsync(g.p, 0, g.bytes, st));
  LYAP_HIP(hipMemsetAsync(c0p.p, 0, c0p.bytes, st));
  LYAP_HIP(hipMemcpyAsync(sig.p, sig_h.data(), P * sizeof(double), hipMemcpyHostToDevice, st));
  LYAP_HIP(hipMemcpyAsync(conv.p, conv_h.data(), P * sizeof(int), hipMemcpyHostToDevice, st));
  // c0 in physical coordinates (V^T X0 = c0 Tout), then v_0 = c0 / beta
  gemm64_rm(sd->c0.as<double>(), ld, sd->Tout.as<double>(), ld, c0p.as<double>(), ld, 1, ld, ld, n,
            st);
  DevBuf beta(sizeof(double));
  hipLaunchKernelGGL(k_sh_normalize, dim3(1), dim3(NT), 0, st, c0p.as<double>(), (int)n,
                     beta.as<double>(), V.as<double>());
  LYAP_HIP(hipGetLastError());
  double beta_h = 0.0;
  LYAP_HIP(hipMemcpyAsync(&beta_h, beta.p, sizeof(double), hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipStreamSynchronize(st));
  {
    std::vector<double> g0((size_t)P * (mmax + 1), 0.0);
    for (int64_t p = 0; p < P; ++p) g0[(size_t)p] = beta_h;  // element 0 of every shift
    LYAP_HIP(hipMemcpyAsync(g.p, g0.data(), g.bytes, hipMemcpyHostToDevice, st));
    LYAP_HIP(hipStreamSynchronize(st));  // g0 is read by the copy until it completes
  }
  const int sgrid = (int)((P + NT - 1) / NT);
  int steps = 0;
  if (beta_h > 0.0) {
    for (int j = 0; j < mmax; ++j) {
      double* vj = V.as<double>() + (long)j * ld;
      double* hcol = Hb.as<double>() + (long)j * ldh;
      // w = K v_j
      seed_apply64(sd, 1, vj, w.as<double>(), st);
      // CGS2 against v_0 .. v_j, then v_(j+1)
      hipLaunchKernelGGL(k_sh_orth, dim3(1), dim3(OT), 0, st, V.as<double>(), ld, w.as<double>(),
                         (int)n, j, hcol, V.as<double>() + (long)(j + 1) * ld);
      const bool poll = (j % kPollEvery) == kPollEvery - 1 || j == mmax - 1;
      if (poll) LYAP_HIP(hipMemsetAsync(unconv.p, 0, sizeof(int), st));
      hipLaunchKernelGGL(k_sh_shift, dim3(sgrid), dim3(NT), 0, st, hcol, j, sig.as<double>(),
                         (int)P, mmax, cs.as<double>(), sn.as<double>(), g.as<double>(),
                         resid.as<double>(), conv.as<int>(), tol * beta_h, unconv.as<int>(),
                         j == mmax - 1 ? 1 : 0);
      LYAP_HIP(hipGetLastError());
      steps = j + 1;
      if (!poll) continue;
      int left = 0;
      double hsub = 0.0;
      LYAP_HIP(hipMemcpyAsync(&left, unconv.p, sizeof(int), hipMemcpyDeviceToHost, st));
      LYAP_HIP(hipMemcpyAsync(&hsub, hcol + j + 1, sizeof(double), hipMemcpyDeviceToHost, st));
      LYAP_HIP(hipStreamSynchronize(st));
      if (left == 0) break;
      LYAP_REQUIRE(hsub > 0.0, LYAP_E_BREAKDOWN, "Arnoldi breakdown before convergence");
    }
  }
  // solutions: z per shift, then Y = Z V (rows of V are the basis vectors)
  DevBuf x((size_t)P * mmax * sizeof(double)), col((size_t)P * (mmax + 1) * sizeof(double)),
      Z((size_t)P * mpad * sizeof(double)), Yp((size_t)P * ld * sizeof(double)),
      tr(P * sizeof(double));
  hipLaunchKernelGGL(k_sh_solve, dim3(sgrid), dim3(NT), 0, st, Hb.as<double>(), ldh,
                     sig.as<double>(), (int)P, mmax, cs.as<double>(), sn.as<double>(),
                     g.as<double>(), conv.as<int>(), x.as<double>(), col.as<double>(),
                     Z.as<double>(), (int)mpad);
  LYAP_HIP(hipGetLastError());
  gemm64_rm(Z.as<double>(), mpad, V.as<double>(), ld, Yp.as<double>(), ld, P, ld, mpad, ld, st);
  batched_dot(tr.as<double>(), Yp.as<double>(), ld, sd->Gam.as<double>(), ld, 1, (int)P, (int)n,
              sd->t0, 2.0, st);
  if (Y_dev)
    LYAP_HIP(hipMemcpy2DAsync(Y_dev, n * sizeof(double), Yp.p, ld * sizeof(double),
                              n * sizeof(double), P, hipMemcpyDeviceToDevice, st));
  std::vector<double> tr_h(P), res_h(P);
  LYAP_HIP(hipMemcpyAsync(tr_h.data(), tr.p, P * sizeof(double), hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipMemcpyAsync(res_h.data(), resid.p, P * sizeof(double), hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipMemcpyAsync(conv_h.data(), conv.p, P * sizeof(int), hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipStreamSynchronize(st));
  for (int64_t p = 0; p < P; ++p) {
    lyap_result& o = res[p];
    const bool zero = d_host[p] == 0.0;
    const double rr = zero || beta_h == 0.0 ? 0.0 : res_h[p] / beta_h;
    o.status = rr <= tol ? LYAP_OK : LYAP_E_NOCONV;
    o.iters = zero ? 0 : steps;
    o.cycles = 1;
    o.refinements = 0;
    o.rel_residual = rr;
    o.err_est = NAN;  // no estimate for the shifted-family solve
    o.trace = tr_h[p];
  }
}

}  // namespace
}  // namespace lyap

using namespace lyap;

extern "C" {

lyap_status smw_solve_shifted(lyap_seed sd, int64_t P, const double* d_host,
                              const lyap_solve_opts* opts, double* Y_dev, lyap_result* res_host,
                              void* hip_stream) {
  if (!sd) return LYAP_E_INVAL;
  LYAP_TRY(shifted_impl(sd, P, d_host, opts, Y_dev, res_host, (hipStream_t)hip_stream));
  return LYAP_OK;
}

}  // extern "C"
