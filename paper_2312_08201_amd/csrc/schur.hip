// Schur-basis seed solve (fallback when the eigenbasis is ill-conditioned).
//
// With the real Schur form A0 = Z T Z^T, the seed Lyapunov solve of a
// right-hand side R becomes the quasi-triangular equation
//     T Xs + Xs T^T = Cs,   Cs = Z^T R Z,   X = Z Xs Z^T,
// solved by Bartels-Stewart back-substitution (the naive baseline method of
// Section 1 applied to the fixed seed).  Columns are produced from the last
// to the first; column j (or the pair j-1, j of a 2x2 block) satisfies
//     T x_j + x_j T_jj = c_j - sum_{l > j} T_jl x_l,
// a shifted quasi-triangular solve done row by row with 1x1 / 2x2 (or 2x4 /
// 4x4 for a column pair) diagonal systems.  One workgroup per problem; the
// problems of a batch share T.  The right-hand side is dense (Cs given) or
// low-rank symmetric, Cs = F G^T + G F^T with F, G stored as k rows of
// length ld, generated on the fly (it is never stored).
#include <algorithm>
#include <vector>

#include "internal.h"

namespace lyap {

namespace {

constexpr int ST = 256;

// small dense solve M x = b (dim <= 4), partial pivoting, in registers
__device__ inline void small_solve(double* M, double* b, int dim) {
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

struct TriArgs {
  const double* T;    // n x ld row-major (upper quasi-triangular)
  const double* Tt;   // T^T row-major
  double* X;          // per problem: n columns of length ld (column j contiguous)
  long xstride;       // elements between problems in X
  const double* Cd;   // dense right-hand side per problem (row-major, symmetric) or null
  long cstride;
  const double* F;    // low-rank factors: k rows of length ld (shared when fstride == 0)
  long fstride;
  const double* G;    // k rows of length ld per problem
  long gstride;
  int k;
  int n, ld;
  const int* list;    // optional: problem index -> slot (engine list)
  const int* count;   // optional: device count of listed problems
};

// rhs_c[i] = C[c][i] - sum_{l > j} T[c][l] X[l][i]    (C[c][i] = C[i][c])
// Four independent partial sums keep several loads of X in flight.
__device__ inline void form_rhs(const TriArgs& A, const double* Cd, const double* Fs,
                                const double* Gs, const double* Xp, int c, int j, double* out) {
  const int n = A.n, ld = A.ld;
  const double* Trow = A.T + (long)c * ld;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double v;
    if (Cd) {
      v = Cd[(long)c * ld + i];
    } else {
      v = 0.0;
      for (int b = 0; b < A.k; ++b) {
        const double* Fb = Fs + (long)b * ld;
        const double* Gb = Gs + (long)b * ld;
        v += Fb[c] * Gb[i] + Gb[c] * Fb[i];
      }
    }
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int l = j + 1;
    for (; l + 3 < n; l += 4) {
      s0 += Trow[l] * Xp[(long)l * ld + i];
      s1 += Trow[l + 1] * Xp[(long)(l + 1) * ld + i];
      s2 += Trow[l + 2] * Xp[(long)(l + 2) * ld + i];
      s3 += Trow[l + 3] * Xp[(long)(l + 3) * ld + i];
    }
    for (; l < n; ++l) s0 += Trow[l] * Xp[(long)l * ld + i];
    out[i] = v - ((s0 + s1) + (s2 + s3));
  }
}

// Rows q = threadIdx.x + k ST (k < NK) of column c of T (only q < c is used),
// read from T^T so that the loads are coalesced.
template <int NK>
__device__ inline void load_col(const double* Tt, int ld, int c, double (&dst)[NK]) {
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int q = threadIdx.x + k * ST;
    dst[k] = (c >= 0 && q < c) ? Tt[(long)c * ld + q] : 0.0;
  }
}

// One workgroup per problem.  The back-substitution over the rows of a column
// (or column pair) is sequential; each step needs the column of T above the
// current row, which is loaded one step ahead into registers (NK per thread)
// so that its latency overlaps the current step's barrier.
template <int NK>
__global__ void __launch_bounds__(ST) k_trilyap(TriArgs A) {
  extern __shared__ double sh[];
  double* b0 = sh;            // rhs of column j-1 (pairs) / j
  double* b1 = sh + A.ld;     // rhs of column j (pairs)
  __shared__ double xs[4];
  int p = blockIdx.x;
  if (A.count && p >= A.count[0]) return;
  const int slot = A.list ? A.list[p] : p;
  const int n = A.n, ld = A.ld;
  double* Xp = A.X + (long)slot * A.xstride;
  const double* Cd = A.Cd ? A.Cd + (long)slot * A.cstride : nullptr;
  const double* Gs = A.G ? A.G + (long)slot * A.gstride : nullptr;
  const double* Fs = A.F ? A.F + (long)slot * A.fstride : nullptr;
  const double* T = A.T;
  const double* Tt = A.Tt;
  const int tid = threadIdx.x;

  int j = n - 1;
  while (j >= 0) {
    const bool pair = j > 0 && T[(long)j * ld + j - 1] != 0.0;
    // columns i and i-1 of T for the first step, prefetched
    double Pi[NK], Pm[NK];
    load_col<NK>(Tt, ld, n - 1, Pi);
    load_col<NK>(Tt, ld, n - 2, Pm);
    if (!pair) {
      form_rhs(A, Cd, Fs, Gs, Xp, j, j, b0);
      __syncthreads();
      const double sg = T[(long)j * ld + j];
      // (T + sg I) x = b0, back-substitution over row blocks
      int i = n - 1;
      while (i >= 0) {
        const bool rp = i > 0 && T[(long)i * ld + i - 1] != 0.0;
        if (!rp) {
          double Pn[NK];
          load_col<NK>(Tt, ld, i - 2, Pn);
          if (tid == 0) xs[0] = b0[i] / (T[(long)i * ld + i] + sg);
          __syncthreads();
          const double xi = xs[0];
#pragma unroll
          for (int k = 0; k < NK; ++k) {
            const int q = tid + k * ST;
            if (q < i) b0[q] -= Pi[k] * xi;
          }
          if (tid == 0) b0[i] = xi;
          __syncthreads();
#pragma unroll
          for (int k = 0; k < NK; ++k) {
            Pi[k] = Pm[k];
            Pm[k] = Pn[k];
          }
          i -= 1;
        } else {
          double Pn0[NK], Pn1[NK];
          load_col<NK>(Tt, ld, i - 2, Pn0);
          load_col<NK>(Tt, ld, i - 3, Pn1);
          if (tid == 0) {
            double M[16], v[4];
            M[0] = T[(long)(i - 1) * ld + i - 1] + sg;
            M[1] = T[(long)(i - 1) * ld + i];
            M[4] = T[(long)i * ld + i - 1];
            M[5] = T[(long)i * ld + i] + sg;
            v[0] = b0[i - 1];
            v[1] = b0[i];
            small_solve(M, v, 2);
            xs[0] = v[0];
            xs[1] = v[1];
          }
          __syncthreads();
          const double x0 = xs[0], x1 = xs[1];
#pragma unroll
          for (int k = 0; k < NK; ++k) {
            const int q = tid + k * ST;
            if (q < i - 1) b0[q] -= Pm[k] * x0 + Pi[k] * x1;
          }
          if (tid == 0) {
            b0[i - 1] = x0;
            b0[i] = x1;
          }
          __syncthreads();
#pragma unroll
          for (int k = 0; k < NK; ++k) {
            Pi[k] = Pn0[k];
            Pm[k] = Pn1[k];
          }
          i -= 2;
        }
      }
      for (int q = tid; q < n; q += blockDim.x) Xp[(long)j * ld + q] = b0[q];
      __syncthreads();
      j -= 1;
    } else {
      // columns j-1, j coupled by S = T[j-1:j+1, j-1:j+1]:  T X2 + X2 S^T = B2
      form_rhs(A, Cd, Fs, Gs, Xp, j - 1, j, b0);
      form_rhs(A, Cd, Fs, Gs, Xp, j, j, b1);
      __syncthreads();
      const double s00 = T[(long)(j - 1) * ld + j - 1], s01 = T[(long)(j - 1) * ld + j];
      const double s10 = T[(long)j * ld + j - 1], s11 = T[(long)j * ld + j];
      int i = n - 1;
      while (i >= 0) {
        const bool rp = i > 0 && T[(long)i * ld + i - 1] != 0.0;
        if (!rp) {
          double Pn[NK];
          load_col<NK>(Tt, ld, i - 2, Pn);
          // x (1x2) solves t x + x S^T = b  ->  [[t+s00, s01],[s10, t+s11]] x = b
          if (tid == 0) {
            const double t = T[(long)i * ld + i];
            double M[16], v[4];
            M[0] = t + s00;
            M[1] = s01;
            M[4] = s10;
            M[5] = t + s11;
            v[0] = b0[i];
            v[1] = b1[i];
            small_solve(M, v, 2);
            xs[0] = v[0];
            xs[1] = v[1];
          }
          __syncthreads();
          const double xa = xs[0], xb = xs[1];
#pragma unroll
          for (int k = 0; k < NK; ++k) {
            const int q = tid + k * ST;
            if (q < i) {
              b0[q] -= Pi[k] * xa;
              b1[q] -= Pi[k] * xb;
            }
          }
          if (tid == 0) {
            b0[i] = xa;
            b1[i] = xb;
          }
          __syncthreads();
#pragma unroll
          for (int k = 0; k < NK; ++k) {
            Pi[k] = Pm[k];
            Pm[k] = Pn[k];
          }
          i -= 1;
        } else {
          double Pn0[NK], Pn1[NK];
          load_col<NK>(Tt, ld, i - 2, Pn0);
          load_col<NK>(Tt, ld, i - 3, Pn1);
          // 2x2 block of T at rows (i-1, i): (I2 kron T_II + S kron I2) vec(X) = vec(B)
          if (tid == 0) {
            const double t00 = T[(long)(i - 1) * ld + i - 1], t01 = T[(long)(i - 1) * ld + i];
            const double t10 = T[(long)i * ld + i - 1], t11 = T[(long)i * ld + i];
            double M[16] = {t00 + s00, t01, s01, 0.0,  //
                            t10, t11 + s00, 0.0, s01,  //
                            s10, 0.0, t00 + s11, t01,  //
                            0.0, s10, t10, t11 + s11};
            double v[4] = {b0[i - 1], b0[i], b1[i - 1], b1[i]};
            small_solve(M, v, 4);
            xs[0] = v[0];
            xs[1] = v[1];
            xs[2] = v[2];
            xs[3] = v[3];
          }
          __syncthreads();
          const double a0 = xs[0], a1 = xs[1], c0 = xs[2], c1 = xs[3];
#pragma unroll
          for (int k = 0; k < NK; ++k) {
            const int q = tid + k * ST;
            if (q < i - 1) {
              b0[q] -= Pm[k] * a0 + Pi[k] * a1;
              b1[q] -= Pm[k] * c0 + Pi[k] * c1;
            }
          }
          if (tid == 0) {
            b0[i - 1] = a0;
            b0[i] = a1;
            b1[i - 1] = c0;
            b1[i] = c1;
          }
          __syncthreads();
#pragma unroll
          for (int k = 0; k < NK; ++k) {
            Pi[k] = Pn0[k];
            Pm[k] = Pn1[k];
          }
          i -= 2;
        }
      }
      for (int q = tid; q < n; q += blockDim.x) {
        Xp[(long)(j - 1) * ld + q] = b0[q];
        Xp[(long)j * ld + q] = b1[q];
      }
      __syncthreads();
      j -= 2;
    }
  }
}

// out[a][:] (row stride ld) = sum_m Vt[a][m] X[m][:]   (X symmetric: column m = row m)
__global__ void k_project(const double* __restrict__ Vt, const double* __restrict__ X, long xstride,
                          double* __restrict__ out, long ostride, int r, int n, int ld,
                          const int* list, const int* count) {
  const int p = blockIdx.y;
  if (count && p >= count[0]) return;
  const int slot = list ? list[p] : p;
  const double* Xp = X + (long)slot * xstride;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int a = 0; a < r; ++a) {
    const double* va = Vt + (long)a * ld;
    double s = 0.0;
    for (int m = 0; m < n; ++m) s += va[m] * Xp[(long)m * ld + i];
    out[(long)slot * ostride + (long)a * ld + i] = s;
  }
}

}  // namespace

void trilyap_launch(const double* T, const double* Tt, double* X, long xstride, const double* Cd,
                    long cstride, const double* F, const double* G, long gstride, int k, int n,
                    int ld, int count, const int* list, const int* count_dev, hipStream_t st,
                    long fstride) {
  TriArgs A{T, Tt, X, xstride, Cd, cstride, F, fstride, G, gstride, k, n, ld, list, count_dev};
  const size_t lds = 2 * (size_t)ld * sizeof(double);
  LYAP_REQUIRE(lds <= 64 * 1024, LYAP_E_INVAL, "Schur-basis solve limited to n <= 4096");
  // rows per thread of a prefetched column: ceil(ld / ST), rounded up to a power of two
  const int nk = (int)((ld + ST - 1) / ST);
  if (nk <= 1) hipLaunchKernelGGL(k_trilyap<1>, dim3(count), dim3(ST), lds, st, A);
  else if (nk <= 2) hipLaunchKernelGGL(k_trilyap<2>, dim3(count), dim3(ST), lds, st, A);
  else if (nk <= 4) hipLaunchKernelGGL(k_trilyap<4>, dim3(count), dim3(ST), lds, st, A);
  else if (nk <= 8) hipLaunchKernelGGL(k_trilyap<8>, dim3(count), dim3(ST), lds, st, A);
  else hipLaunchKernelGGL(k_trilyap<16>, dim3(count), dim3(ST), lds, st, A);
  LYAP_HIP(hipGetLastError());
}

// Dense capacitance operator of a Schur-basis seed.  The map
//     Ys -> Vs^T Xs,   T Xs + Xs T^T = Us Ys + Ys^T Us^T   (Ys: r x n)
// is linear and p-independent.  Row u = b ld + k of Kd (r ld x r ld) is its
// value on the unit input Ys = e_b e_k^T, from one quasi-triangular solve per
// unit input in the orthogonal Schur basis; an engine step is then one GEMM
// z Kd over the active slots.
void schur_dense_operator(lyap_seed_s* sd, hipStream_t st) {
  const long n = sd->n, r = sd->r, ld = sd->ld, rl = r * ld;
  sd->Kd.alloc((size_t)rl * rl * sizeof(double));
  LYAP_HIP(hipMemsetAsync(sd->Kd.p, 0, sd->Kd.bytes, st));
  // unit rows e_k (k < n), the per-problem G factors
  std::vector<double> eye_h((size_t)n * ld, 0.0);
  for (long k = 0; k < n; ++k) eye_h[(size_t)k * ld + k] = 1.0;
  DevBuf eye(eye_h.size() * sizeof(double));
  LYAP_HIP(hipMemcpyAsync(eye.p, eye_h.data(), eye.bytes, hipMemcpyHostToDevice, st));
  // unit problems per launch: enough workgroups to fill the chip, within 16 GiB of solutions
  const long per = (long)ld * ld;
  const long chunk = std::max<long>(1, std::min<long>(n, (long)((size_t(16) << 30) / (per * sizeof(double)))));
  DevBuf Xb((size_t)chunk * per * sizeof(double));
  for (long b = 0; b < r; ++b)
    for (long k0 = 0; k0 < n; k0 += chunk) {
      const int cnt = (int)std::min(chunk, n - k0);
      trilyap_launch(sd->T.as<double>(), sd->Tt.as<double>(), Xb.as<double>(), per, nullptr, 0,
                     sd->Uh.as<double>() + b * ld, eye.as<double>() + k0 * ld, ld, 1, (int)n,
                     (int)ld, cnt, nullptr, nullptr, st);
      project_launch(sd->Vh.as<double>(), Xb.as<double>(), per,
                     sd->Kd.as<double>() + (size_t)(b * ld + k0) * rl, rl, (int)r, (int)n, (int)ld,
                     cnt, nullptr, nullptr, st);
    }
  LYAP_HIP(hipStreamSynchronize(st));
}

void project_launch(const double* Vt, const double* X, long xstride, double* out, long ostride,
                    int r, int n, int ld, int count, const int* list, const int* count_dev,
                    hipStream_t st) {
  dim3 grid((n + 255) / 256, count);
  hipLaunchKernelGGL(k_project, grid, dim3(256), 0, st, Vt, X, xstride, out, ostride, r, n, ld, list,
                     count_dev);
  LYAP_HIP(hipGetLastError());
}

}  // namespace lyap
