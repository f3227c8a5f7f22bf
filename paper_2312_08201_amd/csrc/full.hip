// Full solutions X(p) for functionals other than the trace (the explicit form
// of eq:Xsmalllastline, O(n^3) per parameter):
//     X(p) = X0 + L^-1(U Y + Y^T U^T),   Y = D V^T X(p) from smw_solve_batch,
// i.e. A0 X + X A0^T = -B B^T + U Y + Y^T U^T, one seed Lyapunov solve with a
// right-hand side of rank s + 2r.
//
// Eigen basis.  With the real eigenvector matrix S (pairs as Re/Im columns),
// S^-1 A0 S = Lambda is block diagonal (1x1 real eigenvalues, 2x2 blocks
// [[a, b], [-b, a]] for a +- ib), and Xt = S^-1 X S^-T solves
// Lambda Xt + Xt Lambda^T = S^-1 C S^-T block by block: every pair of blocks
// is an independent linear system of size at most 4.  The seed's rho-vectors
// are these real coordinates scaled by sig (rho(x Q0^-T) = (x S^-T) o sig), and
// Tout = diag(1/sig) S^T, so X = Tout^T Xh Tout with Xh_ij = Xt_ij sig_i sig_j:
// two MFMA GEMMs per parameter after the elementwise solve.
//
// Schur basis.  Xs = Z^T X Z from the batched quasi-triangular solve with the
// low-rank right-hand side [Us, Bs] [Ys, -Bs/2]^T + transpose, then
// X = Z Xs Z^T = Tout^T Xs Tout with the same two GEMMs.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace lyap {
namespace {

constexpr size_t kFullScratch = size_t(3) << 30;  // bytes of per-chunk work buffers

__device__ inline void solve_small(double* M, double* b, int dim) {
  for (int c = 0; c < dim; ++c) {
    int p = c;
    for (int i = c + 1; i < dim; ++i)
      if (fabs(M[i * 4 + c]) > fabs(M[p * 4 + c])) p = i;
    if (p != c) {
      for (int k = 0; k < dim; ++k) {
        const double t = M[c * 4 + k];
        M[c * 4 + k] = M[p * 4 + k];
        M[p * 4 + k] = t;
      }
      const double t = b[c];
      b[c] = b[p];
      b[p] = t;
    }
    const double inv = 1.0 / M[c * 4 + c];
    for (int i = c + 1; i < dim; ++i) {
      const double f = M[i * 4 + c] * inv;
      for (int k = c; k < dim; ++k) M[i * 4 + k] -= f * M[c * 4 + k];
      b[i] -= f * b[c];
    }
  }
  for (int c = dim - 1; c >= 0; --c) {
    double v = b[c];
    for (int k = c + 1; k < dim; ++k) v -= M[c * 4 + k] * b[k];
    b[c] = v / M[c * 4 + c];
  }
}

__device__ inline double sig_of(int q, int h) { return q < 2 * h ? ((q & 1) ? -0.5 : 0.5) : 1.0; }

// One thread per pair of diagonal blocks (I, J) of one parameter (blockIdx.y).
// Right-hand side in real eigen coordinates:
//   C_ij = sum_b (u_b[i] w_b[j] + w_b[i] u_b[j]) - sum_c bt_c[i] bt_c[j]
// with u = Uh / sig, w = Yh / sig, bt = Bh / sig (rows of length ld).
__global__ void k_full_blockdiag(const double* __restrict__ Uh, const double* __restrict__ Yh,
                                 const double* __restrict__ Bh, const double* __restrict__ lam,
                                 double* __restrict__ Xh, int r, int s, int n, int h, int ld,
                                 bool with_y) {
  const int nb = h + (n - 2 * h);
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)nb * nb) return;
  const int p = blockIdx.y;
  const int I = (int)(t / nb), J = (int)(t % nb);
  const int i0 = I < h ? 2 * I : 2 * h + (I - h), mi = I < h ? 2 : 1;
  const int j0 = J < h ? 2 * J : 2 * h + (J - h), mj = J < h ? 2 : 1;
  const double* W = Yh + (long)p * r * ld;
  double c[2][2];
  for (int a = 0; a < mi; ++a)
    for (int e = 0; e < mj; ++e) {
      const int i = i0 + a, j = j0 + e;
      const double si = sig_of(i, h), sj = sig_of(j, h);
      double v = 0.0;
      for (int k = 0; k < s; ++k) v -= (Bh[(long)k * ld + i] / si) * (Bh[(long)k * ld + j] / sj);
      if (with_y)
        for (int b = 0; b < r; ++b)
          v += (Uh[(long)b * ld + i] / si) * (W[(long)b * ld + j] / sj) +
               (W[(long)b * ld + i] / si) * (Uh[(long)b * ld + j] / sj);
      c[a][e] = v;
    }
  // Lambda blocks
  double LI[2][2], LJ[2][2];
  {
    const double a = lam[i0], b = lam[ld + i0];
    LI[0][0] = a; LI[0][1] = b; LI[1][0] = -b; LI[1][1] = a;
  }
  {
    const double a = lam[j0], b = lam[ld + j0];
    LJ[0][0] = a; LJ[0][1] = b; LJ[1][0] = -b; LJ[1][1] = a;
  }
  // (I kron LI + LJ kron I) vec(X) = vec(C), vec column-major: index e * mi + a
  const int dim = mi * mj;
  double M[16], v[4];
  for (int q = 0; q < 16; ++q) M[q] = 0.0;
  for (int e = 0; e < mj; ++e)
    for (int a = 0; a < mi; ++a) {
      const int row = e * mi + a;
      v[row] = c[a][e];
      for (int e2 = 0; e2 < mj; ++e2)
        for (int a2 = 0; a2 < mi; ++a2) {
          const int col = e2 * mi + a2;
          double m = 0.0;
          if (e == e2) m += (mi == 2 ? LI[a][a2] : (a == a2 ? LI[0][0] : 0.0));
          if (a == a2) m += (mj == 2 ? LJ[e][e2] : (e == e2 ? LJ[0][0] : 0.0));
          M[row * 4 + col] = m;
        }
    }
  solve_small(M, v, dim);
  double* X = Xh + (long)p * ld * ld;
  for (int e = 0; e < mj; ++e)
    for (int a = 0; a < mi; ++a) {
      const int i = i0 + a, j = j0 + e;
      X[(long)i * ld + j] = v[e * mi + a] * sig_of(i, h) * sig_of(j, h);
    }
}

// Dense right-hand side in real eigen coordinates (no sig scaling), one thread
// per pair of diagonal blocks (I, J), in place:
//   adjoint = false:  Lambda_I X_IJ + X_IJ Lambda_J^T = C_IJ
//   adjoint = true:   Lambda_I^T X_IJ + X_IJ Lambda_J = C_IJ
__global__ void k_blockdiag_dense(double* __restrict__ C, const double* __restrict__ lam, int n,
                                  int h, int ld, bool adjoint) {
  const int nb = h + (n - 2 * h);
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)nb * nb) return;
  const int I = (int)(t / nb), J = (int)(t % nb);
  const int i0 = I < h ? 2 * I : 2 * h + (I - h), mi = I < h ? 2 : 1;
  const int j0 = J < h ? 2 * J : 2 * h + (J - h), mj = J < h ? 2 : 1;
  const double sgn = adjoint ? -1.0 : 1.0;  // the transposed 2x2 block flips the sign of b
  double LI[2][2], LJ[2][2];
  {
    const double a = lam[i0], b = sgn * lam[ld + i0];
    LI[0][0] = a; LI[0][1] = b; LI[1][0] = -b; LI[1][1] = a;
  }
  {
    // Lambda_J^T (or, for the adjoint, Lambda_J) multiplies from the right:
    // X Lambda_J^T has entries sum_e2 X[a][e2] Lambda_J[e][e2]
    const double a = lam[j0], b = sgn * lam[ld + j0];
    LJ[0][0] = a; LJ[0][1] = b; LJ[1][0] = -b; LJ[1][1] = a;
  }
  const int dim = mi * mj;
  double M[16], v[4];
  for (int q = 0; q < 16; ++q) M[q] = 0.0;
  for (int e = 0; e < mj; ++e)
    for (int a = 0; a < mi; ++a) {
      const int row = e * mi + a;
      v[row] = C[(long)(i0 + a) * ld + (j0 + e)];
      for (int e2 = 0; e2 < mj; ++e2)
        for (int a2 = 0; a2 < mi; ++a2) {
          const int col = e2 * mi + a2;
          double m = 0.0;
          if (e == e2) m += (mi == 2 ? LI[a][a2] : (a == a2 ? LI[0][0] : 0.0));
          if (a == a2) m += (mj == 2 ? LJ[e][e2] : (e == e2 ? LJ[0][0] : 0.0));
          M[row * 4 + col] = m;
        }
    }
  solve_small(M, v, dim);
  for (int e = 0; e < mj; ++e)
    for (int a = 0; a < mi; ++a) C[(long)(i0 + a) * ld + (j0 + e)] = v[e * mi + a];
}

// out = alpha (M + M^T) + beta C on the leading n x n block (C may be null);
// entries outside it are set to zero.
__global__ void k_sym_combine(double* __restrict__ out, const double* __restrict__ M,
                              const double* __restrict__ C, double alpha, double beta, int n,
                              int ld) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)ld * ld) return;
  const int i = (int)(t / ld), j = (int)(t % ld);
  double v = 0.0;
  if (i < n && j < n) {
    v = alpha * (M[(long)i * ld + j] + M[(long)j * ld + i]);
    if (C) v += beta * C[(long)i * ld + j];
  }
  out[t] = v;
}

// out = a + b elementwise over ld x ld
__global__ void k_add(double* __restrict__ out, const double* __restrict__ a,
                      const double* __restrict__ b, long count) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) out[t] = a[t] + b[t];
}

// G rows of the Schur-basis problems: [Ys_p (r rows), -Bs/2 (s rows)]
__global__ void k_full_schur_g(const double* __restrict__ Ys, const double* __restrict__ Bh,
                               double* __restrict__ G, int r, int s, int ld, bool with_y) {
  const int p = blockIdx.y;
  const int k = r + s;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < (long)k * ld;
       e += (long)gridDim.x * blockDim.x) {
    const int row = (int)(e / ld), col = (int)(e % ld);
    double v;
    if (row < r) v = with_y ? Ys[((long)p * r + row) * ld + col] : 0.0;
    else v = -0.5 * Bh[(long)(row - r) * ld + col];
    G[(long)p * k * ld + e] = v;
  }
}

// out_p = in_p^T for count square ld x ld matrices
__global__ void k_transpose_batch(const double* __restrict__ in, double* __restrict__ out, int ld) {
  __shared__ double tile[32][33];
  const long base = (long)blockIdx.z * ld * ld;
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  for (int k = threadIdx.y; k < 32; k += 8) tile[k][threadIdx.x] = in[base + (long)(r0 + k) * ld + c0 + threadIdx.x];
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += 8)
    out[base + (long)(c0 + k) * ld + r0 + threadIdx.x] = tile[threadIdx.x][k];
}

__global__ void k_pad_rows_full(double* __restrict__ dst, long ldd, const double* __restrict__ src,
                                long lds_, int n) {
  const int row = blockIdx.y;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    dst[(long)row * ldd + k] = src[(long)row * lds_ + k];
}

void full_impl(lyap_seed_s* sd, int64_t P, const double* Y, double* X, hipStream_t st) {
  LYAP_REQUIRE(P >= 1 && X, LYAP_E_INVAL, "bad argument");
  LYAP_REQUIRE(Y || P == 1, LYAP_E_INVAL, "without Y only X0 (P = 1) is returned");
  LYAP_REQUIRE(!sd->projected && sd->Bh.p, LYAP_E_UNSUPPORTED,
               "a projected seed holds no right-hand side B");
  const long n = sd->n, ld = sd->ld, r = sd->r, s = sd->s, h = sd->h;
  const bool schur = sd->basis == LYAP_BASIS_SCHUR;
  const size_t mat = (size_t)ld * ld * sizeof(double);
  const long chunk = std::max<long>(1, (long)(kFullScratch / (3 * mat)));
  const size_t rowb = (size_t)ld * sizeof(double);
  for (int64_t p0 = 0; p0 < P; p0 += chunk) {
    const int cnt = (int)std::min<int64_t>(chunk, P - p0);
    DevBuf Yp((size_t)cnt * r * rowb), Yh((size_t)cnt * r * rowb), Xh(cnt * mat), Z(cnt * mat),
        Zt(cnt * mat);
    LYAP_HIP(hipMemsetAsync(Yp.p, 0, Yp.bytes, st));
    LYAP_HIP(hipMemsetAsync(Yh.p, 0, Yh.bytes, st));
    LYAP_HIP(hipMemsetAsync(Xh.p, 0, Xh.bytes, st));
    if (Y) {
      const int ub = (int)std::min<long>((n + 255) / 256, 64);
      hipLaunchKernelGGL(k_pad_rows_full, dim3(ub, (unsigned)(cnt * r)), dim3(256), 0, st,
                         Yp.as<double>(), ld, Y + (size_t)p0 * r * n, n, (int)n);
      LYAP_HIP(hipGetLastError());
      // into the basis: rho(Y Q0^-T) = Y Tin (eigen), Ys = Y Z (Schur)
      gemm64_rm(Yp.as<double>(), ld, sd->Tin.as<double>(), ld, Yh.as<double>(), ld,
                (long)cnt * r, ld, ld, ld, st);
    }
    if (!schur) {
      const long nb = h + (n - 2 * h);
      dim3 grid((unsigned)((nb * nb + 255) / 256), (unsigned)cnt);
      hipLaunchKernelGGL(k_full_blockdiag, grid, dim3(256), 0, st, sd->Uh.as<double>(),
                         Yh.as<double>(), sd->Bh.as<double>(), sd->lam.as<double>(),
                         Xh.as<double>(), (int)r, (int)s, (int)n, (int)h, (int)ld, Y != nullptr);
      LYAP_HIP(hipGetLastError());
    } else {
      const long k = r + s;
      DevBuf F((size_t)k * rowb), G((size_t)cnt * k * rowb);
      LYAP_HIP(hipMemcpyAsync(F.p, sd->Uh.p, (size_t)r * rowb, hipMemcpyDeviceToDevice, st));
      LYAP_HIP(hipMemcpyAsync(F.as<double>() + r * ld, sd->Bh.p, (size_t)s * rowb,
                              hipMemcpyDeviceToDevice, st));
      hipLaunchKernelGGL(k_full_schur_g, dim3(64, (unsigned)cnt), dim3(256), 0, st,
                         Yh.as<double>(), sd->Bh.as<double>(), G.as<double>(), (int)r, (int)s,
                         (int)ld, Y != nullptr);
      LYAP_HIP(hipGetLastError());
      trilyap_blocked(sd->T.as<double>(), sd->Tt.as<double>(), (int)n, (int)ld, nullptr,
                      F.as<double>(), 0, G.as<double>(), k * ld, (int)k, cnt, ld, Xh.as<double>(),
                      st);
    }
    // X = Tout^T Xh Tout: Z = Xh Tout, then X = Z^T Tout (Xh symmetric)
    gemm64_rm(Xh.as<double>(), ld, sd->Tout.as<double>(), ld, Z.as<double>(), ld, (long)cnt * ld,
              ld, ld, ld, st);
    {
      dim3 grid((unsigned)(ld / 32), (unsigned)(ld / 32), (unsigned)cnt);
      hipLaunchKernelGGL(k_transpose_batch, grid, dim3(32, 8), 0, st, Z.as<double>(),
                         Zt.as<double>(), (int)ld);
      LYAP_HIP(hipGetLastError());
    }
    for (int q = 0; q < cnt; ++q)
      gemm64_rm(Zt.as<double>() + (size_t)q * ld * ld, ld, sd->Tout.as<double>(), ld,
                X + (size_t)(p0 + q) * n * n, n, n, ld, ld, n, st);
    LYAP_HIP(hipStreamSynchronize(st));
  }
}

}  // namespace

void blockdiag_dense_launch(double* C, const double* lam, int n, int h, int ld, bool adjoint,
                            hipStream_t st) {
  const long nb = h + (n - 2 * h);
  hipLaunchKernelGGL(k_blockdiag_dense, dim3((unsigned)((nb * nb + 255) / 256)), dim3(256), 0, st,
                     C, lam, n, h, ld, adjoint);
  LYAP_HIP(hipGetLastError());
}

void sym_combine_launch(double* out, const double* M, const double* C, double alpha, double beta,
                        int n, int ld, hipStream_t st) {
  const long cnt = (long)ld * ld;
  hipLaunchKernelGGL(k_sym_combine, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, out, M,
                     C, alpha, beta, n, ld);
  LYAP_HIP(hipGetLastError());
}

void add_launch(double* out, const double* a, const double* b, long count, hipStream_t st) {
  hipLaunchKernelGGL(k_add, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, out, a, b,
                     count);
  LYAP_HIP(hipGetLastError());
}

}  // namespace lyap

using namespace lyap;

extern "C" {

lyap_status seed_full_X(lyap_seed sd, int64_t P, const double* Y_dev, double* X_dev,
                        void* hip_stream) {
  if (!sd) return LYAP_E_INVAL;
  LYAP_TRY(full_impl(sd, P, Y_dev, X_dev, (hipStream_t)hip_stream));
  return LYAP_OK;
}

}  // extern "C"
