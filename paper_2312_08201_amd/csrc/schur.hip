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

// ---------------------------------------------------------------------------
// Tile-blocked back-substitution for a batch of problems sharing T.
// Problem b (X_b row-major, n rows of ld, problems n ld apart) solves
//     T X_b + X_b T^T = F G_b^T + G_b F^T.
// Column panels J (width <= kPanel) are produced from the last to the first,
// and inside a panel the row tiles I (height <= kTile) from the bottom up.
// Tile (I, J) satisfies
//     T_II X_IJ + X_IJ T_JJ^T = C_IJ - sum_{L > J} X_IL T_JL^T - sum_{K > I} T_IK X_KJ.
// The first sum, for a whole panel and every problem, is one GEMM (the solved
// columns of all problems stacked as rows, times T^T); the second, for one
// tile row, is one GEMM of T's rows with the solved rows of the panel, kept
// problem-interleaved as Panel[k][b][j].  Both read their K range from a
// 16-aligned start: the entries in front of the true start belong to the
// tile being solved and are still zero.  No 2x2 block of T straddles a tile
// boundary.  The tile equation is solved by one wavefront per problem: lane
// q owns row q, the columns go from the last to the first (column pairs for
// 2x2 blocks of T_JJ) and the rows of each column from the bottom up, the
// solved entry being broadcast with readlane.
constexpr int kTile = 64;     // row tile height = lanes of the tile kernel
constexpr int kPanel = 120;   // column panel width (GEMM N tile is 128)
constexpr int kXs = kPanel + 1;

struct TileArgs {
  const double* T;    // n x ld row-major
  int n, ld;
  int I0, ni, J0, nj;
  const double* Cd;   // dense symmetric right-hand side (row-major, ld), or null
  const double* F;    // k rows of ld (shared when fstride == 0)
  long fstride;
  const double* G;    // k rows of ld per problem (shared when gstride == 0)
  long gstride;
  int k;
  const double* P;    // (problems xrows) x 128: sum_{L > J} X_IL T_JL^T, or null
  const double* Q;    // ni x npad: sum_{K > I} T_IK X_KJ, column b kPanel + j, or null
  long npad;
  double* X;          // problems xrows ld apart
  long xrows;
  double* Panel;      // kend x npad: solved rows of the panel, column b kPanel + j
};

__device__ inline double readlane_d(double v, int l) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// inverse of a D x D matrix (D <= 4, row-major, stride 4) by Gauss-Jordan
// elimination with partial pivoting, into R (row-major, stride 4).  All
// indices are compile-time (pivot rows are exchanged by conditional swaps),
// so the arrays stay in registers without indexed moves.
template <int D>
__device__ inline void small_inverse(double (&M)[16], double (&R)[16]) {
#pragma unroll
  for (int e = 0; e < 16; ++e) R[e] = (e % 5 == 0) ? 1.0 : 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
#pragma unroll
    for (int i = c + 1; i < D; ++i) {
      const bool sw = fabs(M[i * 4 + c]) > fabs(M[c * 4 + c]);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double mc = M[c * 4 + k], mi = M[i * 4 + k];
        M[c * 4 + k] = sw ? mi : mc;
        M[i * 4 + k] = sw ? mc : mi;
        const double rc = R[c * 4 + k], ri = R[i * 4 + k];
        R[c * 4 + k] = sw ? ri : rc;
        R[i * 4 + k] = sw ? rc : ri;
      }
    }
    const double inv = 1.0 / M[c * 4 + c];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      M[c * 4 + k] *= inv;
      R[c * 4 + k] *= inv;
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
      if (i == c) continue;
      const double f = M[i * 4 + c];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        M[i * 4 + k] -= f * M[c * 4 + k];
        R[i * 4 + k] -= f * R[c * 4 + k];
      }
    }
  }
}

constexpr int kInv = 17;  // LDS stride of a lane's inverse (16 entries)
constexpr int kTs = kTile + 1;

__global__ void __launch_bounds__(kTile) k_tile_lyap(TileArgs A) {
  __shared__ double Xt[kTile * kXs];     // right-hand side, overwritten by the solution
  __shared__ double Minv[kTile * kInv];  // per row block: inverse of its small system
  __shared__ double Ts[kTile * kTs];     // T_II, row q at q kTs
  const int b = blockIdx.x, q = threadIdx.x;
  const int ld = A.ld, I0 = A.I0, ni = A.ni, J0 = A.J0, nj = A.nj;
  const double* T = A.T;
  const bool live = q < ni;
  const int gi = I0 + (live ? q : 0);  // this lane's row of T and X
  double* xrow = Xt + q * kXs;

  // T_II into LDS (row r of the tile, column q; lanes beyond the tile read
  // its first column instead), and the right-hand side's dense and low-rank
  // parts into Xt (columns q and q + 64 of each row).  The GEMM products P
  // and Q are subtracted column by column below, fetched one column step ahead.
  const int c0 = q, c1 = q + 64;
  const bool has0 = c0 < nj, has1 = c1 < nj;
  const int tc = I0 + (live ? q : 0);
#pragma unroll 8
  for (int r = 0; r < ni; ++r) Ts[r * kTs + q] = T[(long)(I0 + r) * ld + tc];
  for (int r = 0; r < ni; ++r) {
    const long g = I0 + r;
    if (has0) Xt[r * kXs + c0] = A.Cd ? A.Cd[g * ld + J0 + c0] : 0.0;
    if (has1) Xt[r * kXs + c1] = A.Cd ? A.Cd[g * ld + J0 + c1] : 0.0;
  }
  for (int t = 0; t < A.k; ++t) {
    const double* Ft = A.F + (long)b * A.fstride + (long)t * ld;
    const double* Gt = A.G + (long)b * A.gstride + (long)t * ld;
    const double f0 = has0 ? Ft[J0 + c0] : 0.0, g0 = has0 ? Gt[J0 + c0] : 0.0;
    const double f1 = has1 ? Ft[J0 + c1] : 0.0, g1 = has1 ? Gt[J0 + c1] : 0.0;
#pragma unroll 8
    for (int r = 0; r < ni; ++r) {
      const double fr = Ft[I0 + r], gr = Gt[I0 + r];
      if (has0) Xt[r * kXs + c0] += fr * g0 + gr * f0;
      if (has1) Xt[r * kXs + c1] += fr * g1 + gr * f1;
    }
  }
  // P + Q at column c of this lane's row, as two loads (summed where used)
  auto load_pq = [&](int c, double& pv, double& qv) {
    const bool ok = live && c >= 0;
    pv = (ok && A.P) ? A.P[((long)b * A.xrows + gi) * 128 + c] : 0.0;
    qv = (ok && A.Q) ? A.Q[(long)q * A.npad + (long)b * kPanel + c] : 0.0;
  };
  // diagonal band of T_II (this lane's row) and of T_JJ (columns q and q + 64)
  const double dI = live ? T[(long)gi * ld + gi] : 1.0;
  const double subI = (live && q > 0) ? T[(long)gi * ld + gi - 1] : 0.0;   // T[q][q-1]
  const double supI = (live && q > 0) ? T[(long)(gi - 1) * ld + gi] : 0.0; // T[q-1][q]
  const double dIp = (live && q > 0) ? T[(long)(gi - 1) * ld + gi - 1] : 0.0;
  const unsigned long long rmask = __ballot(subI != 0.0);  // bit i: rows i-1, i form a 2x2 block
  double dJ[2], subJ[2], supJ[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = q + 64 * h, gc = J0 + c;
    const bool in = c < nj;
    dJ[h] = in ? T[(long)gc * ld + gc] : 0.0;
    subJ[h] = (in && c > 0) ? T[(long)gc * ld + gc - 1] : 0.0;
    supJ[h] = (in && c > 0) ? T[(long)(gc - 1) * ld + gc] : 0.0;
  }
  const unsigned long long cmask0 = __ballot(subJ[0] != 0.0);
  const unsigned long long cmask1 = __ballot(subJ[1] != 0.0);
  auto colv = [&](const double (&v)[2], int c) -> double {
    return c < 64 ? readlane_d(v[0], c) : readlane_d(v[1], c - 64);
  };
  auto cpair_of = [&](int c) -> bool {
    return c > 0 && (c < 64 ? ((cmask0 >> c) & 1ULL) : ((cmask1 >> (c - 64)) & 1ULL));
  };
  const bool rbot = (rmask >> q) & 1ULL;  // this lane ends a 2x2 row block
  // T[gi][I0 + i]: column i of T_II, one row per lane
  const double* trow = Ts + q * kTs;
  __syncthreads();

  // rows c of T_JJ spread over the lanes (lane l: columns l and l + 64)
  auto load_trow = [&](int c, double (&tr)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int cc = q + 64 * h;
      tr[h] = (c >= 0 && cc < nj) ? T[(long)(J0 + c) * ld + J0 + cc] : 0.0;
    }
  };
  int j = nj - 1;
  bool cpair = cpair_of(j);
  int jc = cpair ? j - 1 : j;  // first column of the step
  double trA[2], trB[2];       // rows jc and j of T_JJ
  load_trow(jc, trA);
  load_trow(j, trB);
  double pA, qA, pB, qB;       // P and Q at columns jc and j
  load_pq(jc, pA, qA);
  load_pq(j, pB, qB);
  while (j >= 0) {
    // right-hand sides: the X T_JJ^T sum over the solved columns l > j, in two
    // ranges so that the register holding T_JJ[.][l] is fixed in each loop
    double b0 = 0.0, b1 = 0.0;
    {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      const int mid = nj < 64 ? nj : 64;
      int l = j + 1;
      for (; l + 1 < mid; l += 2) {
        const double x0 = xrow[l], x1 = xrow[l + 1];
        s0 += readlane_d(trA[0], l) * x0;
        s1 += readlane_d(trA[0], l + 1) * x1;
        s2 += readlane_d(trB[0], l) * x0;
        s3 += readlane_d(trB[0], l + 1) * x1;
      }
      for (; l < mid; ++l) {
        const double x0 = xrow[l];
        s0 += readlane_d(trA[0], l) * x0;
        s2 += readlane_d(trB[0], l) * x0;
      }
      for (; l + 1 < nj; l += 2) {
        const double x0 = xrow[l], x1 = xrow[l + 1];
        s0 += readlane_d(trA[1], l - 64) * x0;
        s1 += readlane_d(trA[1], l - 63) * x1;
        s2 += readlane_d(trB[1], l - 64) * x0;
        s3 += readlane_d(trB[1], l - 63) * x1;
      }
      for (; l < nj; ++l) {
        const double x0 = xrow[l];
        s0 += readlane_d(trA[1], l - 64) * x0;
        s2 += readlane_d(trB[1], l - 64) * x0;
      }
      if (live) {
        b0 = ((xrow[jc] - pA) - qA) - (s0 + s1);
        b1 = ((xrow[j] - pB) - qB) - (s2 + s3);
      }
    }
    // the next step's rows, loaded now so that the substitution below hides them
    const int jn = jc - 1;
    const bool cpn = cpair_of(jn);
    const int jcn = cpn ? jn - 1 : jn;
    double tnA[2], tnB[2];
    load_trow(jcn, tnA);
    load_trow(jn, tnB);
    double pAn, qAn, pBn, qBn;
    load_pq(jcn, pAn, qAn);
    load_pq(jn, pBn, qBn);
    // each row block's small system, inverted by the lane that ends the block
    {
      double M[16], R[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) M[e] = 0.0;
      if (!cpair) {
        const double sg = colv(dJ, j);
        if (!rbot) {
          M[0] = dI + sg;
          small_inverse<1>(M, R);
        } else {
          M[0] = dIp + sg;
          M[1] = supI;
          M[4] = subI;
          M[5] = dI + sg;
          small_inverse<2>(M, R);
        }
      } else {
        const double s00 = colv(dJ, j - 1), s01 = colv(supJ, j);
        const double s10 = colv(subJ, j), s11 = colv(dJ, j);
        if (!rbot) {
          M[0] = dI + s00;
          M[1] = s01;
          M[4] = s10;
          M[5] = dI + s11;
          small_inverse<2>(M, R);
        } else {
          // unknowns (x[i-1][j-1], x[i][j-1], x[i-1][j], x[i][j])
          const double t00 = dIp, t01 = supI, t10 = subI, t11 = dI;
          M[0] = t00 + s00; M[1] = t01;       M[2] = s01;        M[3] = 0.0;
          M[4] = t10;       M[5] = t11 + s00; M[6] = 0.0;        M[7] = s01;
          M[8] = s10;       M[9] = 0.0;       M[10] = t00 + s11; M[11] = t01;
          M[12] = 0.0;      M[13] = s10;      M[14] = t10;       M[15] = t11 + s11;
          small_inverse<4>(M, R);
        }
      }
#pragma unroll
      for (int e = 0; e < 16; ++e) Minv[q * kInv + e] = R[e];
    }
    __syncthreads();
    // back-substitution over the rows (lanes q < i update with T[q][i])
    int i = ni - 1;
    while (i >= 0) {
      const bool rpair = (rmask >> i) & 1ULL;
      const double* Mi = Minv + i * kInv;
      const double w0 = trow[i];
      if (!rpair) {
        if (!cpair) {
          const double x = readlane_d(b0, i) * Mi[0];
          if (q < i) b0 -= w0 * x;
          else if (q == i) b0 = x;
        } else {
          const double u0 = readlane_d(b0, i), u1 = readlane_d(b1, i);
          const double xa = Mi[0] * u0 + Mi[1] * u1;
          const double xb = Mi[4] * u0 + Mi[5] * u1;
          if (q < i) {
            b0 -= w0 * xa;
            b1 -= w0 * xb;
          } else if (q == i) {
            b0 = xa;
            b1 = xb;
          }
        }
        i -= 1;
      } else {
        const double w1 = trow[i - 1];
        if (!cpair) {
          const double u0 = readlane_d(b0, i - 1), u1 = readlane_d(b0, i);
          const double x0 = Mi[0] * u0 + Mi[1] * u1;
          const double x1 = Mi[4] * u0 + Mi[5] * u1;
          if (q < i - 1) b0 -= w1 * x0 + w0 * x1;
          else if (q == i - 1) b0 = x0;
          else if (q == i) b0 = x1;
        } else {
          const double u0 = readlane_d(b0, i - 1), u1 = readlane_d(b0, i);
          const double u2 = readlane_d(b1, i - 1), u3 = readlane_d(b1, i);
          const double v0 = Mi[0] * u0 + Mi[1] * u1 + Mi[2] * u2 + Mi[3] * u3;
          const double v1 = Mi[4] * u0 + Mi[5] * u1 + Mi[6] * u2 + Mi[7] * u3;
          const double v2 = Mi[8] * u0 + Mi[9] * u1 + Mi[10] * u2 + Mi[11] * u3;
          const double v3 = Mi[12] * u0 + Mi[13] * u1 + Mi[14] * u2 + Mi[15] * u3;
          if (q < i - 1) {
            b0 -= w1 * v0 + w0 * v1;
            b1 -= w1 * v2 + w0 * v3;
          } else if (q == i - 1) {
            b0 = v0;
            b1 = v2;
          } else if (q == i) {
            b0 = v1;
            b1 = v3;
          }
        }
        i -= 2;
      }
    }
    if (live) {
      xrow[jc] = b0;
      if (cpair) xrow[j] = b1;
    }
    __syncthreads();  // Minv is rewritten by the next column step
    j = jn;
    cpair = cpn;
    jc = jcn;
    pA = pAn;
    qA = qAn;
    pB = pBn;
    qB = qBn;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      trA[h] = tnA[h];
      trB[h] = tnB[h];
    }
  }
  // write the tile row by row (coalesced over the columns)
  double* Xb = A.X + (long)b * A.xrows * ld;
  for (int r = 0; r < ni; ++r) {
    const int g = I0 + r;
    for (int c = q; c < nj; c += kTile) {
      const double v = Xt[r * kXs + c];
      Xb[(long)g * ld + J0 + c] = v;
      A.Panel[(long)g * A.npad + (long)b * kPanel + c] = v;
    }
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

namespace {

// sub[i - 1] = T[i][i - 1], 0 < i < n
__global__ void k_subdiag(const double* __restrict__ T, int ld, int n, double* __restrict__ sub) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
  if (i < n) sub[i - 1] = T[(long)i * ld + i - 1];
}

// Tile boundaries 0 = b_0 < ... < b_m = n of nominal size nb, from the bottom
// up, moved down by one row where a 2x2 block would straddle (sub[i - 1] =
// T[i][i - 1]).
std::vector<int> schur_bounds(const std::vector<double>& sub, int n, int nb) {
  std::vector<int> b{n};
  while (b.back() > 0) {
    int nx = b.back() - nb;
    if (nx <= 0) {
      b.push_back(0);
      break;
    }
    if (sub[nx - 1] != 0.0) nx += 1;
    b.push_back(nx);
  }
  std::reverse(b.begin(), b.end());
  return b;
}

long pad16(long v) { return (v + 15) / 16 * 16; }

// Batched blocked solver for one quasi-triangular T (see k_tile_lyap).
struct BlockedLyap {
  const double* T;
  const double* Tt;
  int n, ld;
  long kend, ldt;
  std::vector<int> rb, cb;
  DevBuf Ttp;  // T^T with 128 zero columns appended, so a 128-column GEMM tile never leaves it

  BlockedLyap(const double* T_, const double* Tt_, int n_, int ld_, hipStream_t st)
      : T(T_), Tt(Tt_), n(n_), ld(ld_), kend(pad16(n_)), ldt(ld_ + 128) {
    LYAP_REQUIRE(ld % 16 == 0 && kend <= ld, LYAP_E_INVAL, "blocked Schur solve: bad padding");
    // subdiagonal of T, gathered on the device and copied back contiguously
    std::vector<double> sub(std::max(n - 1, 1), 0.0);
    if (n > 1) {
      DevBuf subd(sub.size() * sizeof(double));
      hipLaunchKernelGGL(k_subdiag, dim3((unsigned)((n - 1 + 255) / 256)), dim3(256), 0, st, T, ld,
                         n, subd.as<double>());
      LYAP_HIP(hipGetLastError());
      LYAP_HIP(hipMemcpyAsync(sub.data(), subd.p, subd.bytes, hipMemcpyDeviceToHost, st));
      LYAP_HIP(hipStreamSynchronize(st));
    }
    Ttp.alloc((size_t)ld * ldt * sizeof(double));
    LYAP_HIP(hipMemsetAsync(Ttp.p, 0, Ttp.bytes, st));
    LYAP_HIP(hipMemcpy2DAsync(Ttp.p, ldt * sizeof(double), Tt, ld * sizeof(double),
                              ld * sizeof(double), ld, hipMemcpyDeviceToDevice, st));
    LYAP_HIP(hipStreamSynchronize(st));
    rb = schur_bounds(sub, n, kTile);
    cb = schur_bounds(sub, n, kPanel);
  }

  long npad(long count) const { return (count * kPanel + 127) / 128 * 128; }
  // device bytes per problem with n rows: X, the panel products P and the panel rows
  size_t bytes_per_problem() const {
    return ((size_t)n * ld + (size_t)n * 128 + (size_t)kend * kPanel + 128) * sizeof(double);
  }

  // X (count problems of xrows >= n rows of ld; rows >= n are zero):
  // T X_b + X_b T^T = Cd + F G_b^T + G_b F^T (Cd shared, or null).
  // Workspace: P count xrows x 128, Panel kend x npad(count), Q kTile x npad(count).
  void solve(const double* Cd, const double* F, long fstride, const double* G, long gstride, int k,
             long count, long xrows, double* X, double* P, double* Panel, double* Q,
             hipStream_t st) const {
    const long np = npad(count);
    LYAP_REQUIRE(xrows >= n && count * xrows < (1L << 31), LYAP_E_INVAL,
                 "blocked Schur solve: batch too large");
    LYAP_HIP(hipMemsetAsync(X, 0, (size_t)count * xrows * ld * sizeof(double), st));
    for (int jb = (int)cb.size() - 2; jb >= 0; --jb) {
      const int J0 = cb[jb], Jend = cb[jb + 1];
      const bool haveP = Jend < n;
      if (haveP) {
        const long ks = Jend / 16 * 16;
        GemmArgs g{};
        g.type = GemmType::F64;
        g.A = X + ks;
        g.lda = ld;
        g.M = count * xrows;
        g.B = Ttp.as<double>() + ks * ldt + J0;
        g.ldb = ldt;
        g.N = 128;
        g.Nstore = 128;
        g.K = kend - ks;
        g.C = P;
        g.ldc = 128;
        gemm_launch(g, st);
      }
      LYAP_HIP(hipMemsetAsync(Panel, 0, (size_t)kend * np * sizeof(double), st));
      for (int ib = (int)rb.size() - 2; ib >= 0; --ib) {
        const int I0 = rb[ib], Iend = rb[ib + 1];
        const bool haveQ = Iend < n;
        if (haveQ) {
          const long ks = Iend / 16 * 16;
          GemmArgs g{};
          g.type = GemmType::F64;
          g.A = T + (long)I0 * ld + ks;
          g.lda = ld;
          g.M = Iend - I0;
          g.B = Panel + ks * np;
          g.ldb = np;
          g.N = np;
          g.Nstore = np;
          g.K = kend - ks;
          g.C = Q;
          g.ldc = np;
          gemm_launch(g, st);
        }
        TileArgs A{T,  n, ld, I0, Iend - I0, J0, Jend - J0, Cd, F, fstride, G, gstride, k,
                   haveP ? P : nullptr, haveQ ? Q : nullptr, np, X, xrows, Panel};
        hipLaunchKernelGGL(k_tile_lyap, dim3((unsigned)count), dim3(kTile), 0, st, A);
        LYAP_HIP(hipGetLastError());
      }
    }
  }
};

}  // namespace

void trilyap_blocked(const double* T, const double* Tt, int n, int ld, const double* Cd,
                     const double* F, long fstride, const double* G, long gstride, int k,
                     long count, long xrows, double* X, hipStream_t st) {
  BlockedLyap bl(T, Tt, n, ld, st);
  DevBuf P((size_t)count * xrows * 128 * sizeof(double));
  DevBuf Panel((size_t)bl.kend * bl.npad(count) * sizeof(double));
  DevBuf Q((size_t)kTile * bl.npad(count) * sizeof(double));
  bl.solve(Cd, F, fstride, G, gstride, k, count, xrows, X, P.as<double>(), Panel.as<double>(),
           Q.as<double>(), st);
  LYAP_HIP(hipStreamSynchronize(st));
}

// Dense capacitance operator of a Schur-basis seed.  The map
//     Ys -> Vs^T Xs,   T Xs + Xs T^T = Us Ys + Ys^T Us^T   (Ys: r x n)
// is linear and p-independent.  Row u = b ld + k of Kd (r ld x r ld) is its
// value on the unit input Ys = e_b e_k^T, from one quasi-triangular solve per
// unit input in the orthogonal Schur basis (the tile-blocked solver, many
// unit inputs per launch); an engine step is then one GEMM z Kd over the
// active slots.
void schur_dense_operator(lyap_seed_s* sd, hipStream_t st) {
  const long n = sd->n, r = sd->r, ld = sd->ld, rl = r * ld;
  sd->Kd.alloc((size_t)rl * rl * sizeof(double));
  LYAP_HIP(hipMemsetAsync(sd->Kd.p, 0, sd->Kd.bytes, st));
  // unit rows e_k (k < n), the per-problem G factors
  std::vector<double> eye_h((size_t)n * ld, 0.0);
  for (long k = 0; k < n; ++k) eye_h[(size_t)k * ld + k] = 1.0;
  DevBuf eye(eye_h.size() * sizeof(double));
  LYAP_HIP(hipMemcpyAsync(eye.p, eye_h.data(), eye.bytes, hipMemcpyHostToDevice, st));
  BlockedLyap bl(sd->T.as<double>(), sd->Tt.as<double>(), (int)n, (int)ld, st);
  // unit problems per launch: within 16 GiB of solutions and workspace
  const long chunk = std::max<long>(
      1, std::min<long>(n, (long)((size_t(16) << 30) / bl.bytes_per_problem())));
  DevBuf Xb((size_t)chunk * n * ld * sizeof(double));
  DevBuf P((size_t)chunk * n * 128 * sizeof(double));
  DevBuf Panel((size_t)bl.kend * bl.npad(chunk) * sizeof(double));
  DevBuf Q((size_t)kTile * bl.npad(chunk) * sizeof(double));
  for (long b = 0; b < r; ++b)
    for (long k0 = 0; k0 < n; k0 += chunk) {
      const long cnt = std::min(chunk, n - k0);
      bl.solve(nullptr, sd->Uh.as<double>() + b * ld, 0, eye.as<double>() + k0 * ld, ld, 1, cnt, n,
               Xb.as<double>(), P.as<double>(), Panel.as<double>(), Q.as<double>(), st);
      project_launch(sd->Vh.as<double>(), Xb.as<double>(), n * ld,
                     sd->Kd.as<double>() + (size_t)(b * ld + k0) * rl, rl, (int)r, (int)n, (int)ld,
                     (int)cnt, nullptr, nullptr, st);
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
