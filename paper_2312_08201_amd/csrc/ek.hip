// Projection framework for large seeds (Section 2.2, Algorithm EKSM_opt).
//
// One extended Krylov space EK_m(A0, P) (eq:EK_def), P = [X0 V, U] the factor
// of the right-hand side of the correction equation (eq:rhs_newexpression),
// serves every parameter.  With an orthonormal basis Q_m of it, the Galerkin
// condition gives the projected equation (eq:param_projected)
//     A_m(d) Y + Y A_m(d)^T = G_m J(d) G_m^T,   A_m(d) = T_m - U_m D V_m^T,
// T_m = Q_m^T A0 Q_m, U_m = Q_m^T U, V_m = Q_m^T V, G_m = Q_m^T P.
// Writing W = D (V_m^T Y + C^T) with C = Q_m^T X0 V turns it into the SMW
// capacitance system of Section 2.1 for the small seed T_m,
//     (I - D K_m) W = D C^T,   K_m(W) = V_m^T L_{T_m}^-1(U_m W + W^T U_m^T),
// so the projected equations of all parameters are solved by the batched
// Krylov engine on a projected seed (factor_projected) whose right-hand side
// enters through C^T and t0 = trace(E X0) only.  f(X) = t0 + trace(E_m Y),
// E_m = Q_m^T E Q_m, is the engine's trace functional of that seed.
//
// Backward error (Proposition on the backward error): with L = Q_(m+1)^T A0 Q_m
// (the coupling to the next block, from A0 Q_m in the span of Q_(m+1)),
//     Delta = sqrt(2) ||L Y||_F / (2 ||A(d)||_F ||Y||_F + ||P J(d) P^T||_F),
//     Y = L_{T_m}^-1(U_m W + W^T U_m^T).
// In the real Schur basis T_m = Z Ts Z^T both norms are orthogonally
// invariant: ||Y||_F = ||Ys||_F and ||L Y||_F = ||(L Z) Ys||_F with
// Ts Ys + Ys Ts^T = Zs^T(...)Z, so each parameter costs one batched
// quasi-triangular solve of the projected size plus two norms.  ||A(d)||_F and
// ||P J P^T||_F come from p-independent r x r tables.
//
// The basis is built on the host (offline stage, like the seed
// factorisation): LU of A0 by LAPACK, blocks [A0 W+, A0^-1 W-] orthogonalised
// twice against the earlier blocks and then column by column, columns that
// fall below a relative 1e-10 dropped (deflation).
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "internal.h"
#include "lapack_host.h"
#include "schur_host.h"

namespace lyap {
namespace {

constexpr double kDeflate = 1e-10;
constexpr int NT = 256;
constexpr int kDeltaChunk = 1024;   // problems per batched quasi-triangular solve
constexpr size_t kOpBytes = size_t(8) << 30;  // temporary bytes allowed for building operators

// dst (rows x ldd) <- src (rows x n), pads untouched (caller zeroes them)
__global__ void k_pad_rows_ek(double* __restrict__ dst, long ldd, const double* __restrict__ src,
                              long lds_, int n) {
  const int row = blockIdx.y;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    dst[(long)row * ldd + k] = src[(long)row * lds_ + k];
}

// One workgroup per parameter: ||Ys||_F, ||Lz Ys||_F and the backward error.
// Ys is symmetric; row i of it is read as column i (coalesced over j).
// cst: [||A0||_F^2, H (r x r), a (r), Gm (2r x 2r)].
__global__ void __launch_bounds__(NT)
k_ek_delta(const double* __restrict__ Xs, long xstride, int n, int ld,
           const double* __restrict__ Lz, int q, const double* __restrict__ d, int r,
           const double* __restrict__ cst, double* __restrict__ delta, double* __restrict__ nrm) {
  const int p = blockIdx.x;
  const double* X = Xs + (long)p * xstride;
  double sy = 0.0, sr = 0.0;
  for (int j = threadIdx.x; j < n; j += NT) {
    for (int i = 0; i < n; ++i) {
      const double x = X[(long)i * ld + j];
      sy += x * x;
    }
    for (int a0 = 0; a0 < q; a0 += 8) {
      double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      const int na = min(8, q - a0);
      for (int i = 0; i < n; ++i) {
        const double x = X[(long)i * ld + j];
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (t < na) acc[t] += Lz[(long)(a0 + t) * ld + i] * x;
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) sr += acc[t] * acc[t];
    }
  }
  __shared__ double red[2][NT];
  red[0][threadIdx.x] = sy;
  red[1][threadIdx.x] = sr;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double* dp = d + (long)p * r;
    const double* H = cst + 1;
    const double* av = H + r * r;
    const double* Gm = av + r;
    double a2 = cst[0];
    for (int i = 0; i < r; ++i) {
      a2 -= 2.0 * av[i] * dp[i];
      for (int j = 0; j < r; ++j) a2 += dp[i] * dp[j] * H[i * r + j];
    }
    // ||P J P^T||_F^2 = trace(J Gm J Gm), J = [[0, D], [D, 0]]
    const int r2 = 2 * r;
    double g2 = 0.0;
    for (int a = 0; a < r2; ++a)
      for (int c = 0; c < r2; ++c) {
        const double mac = (a < r ? dp[a] * Gm[(a + r) * r2 + c] : dp[a - r] * Gm[(a - r) * r2 + c]);
        const double mca = (c < r ? dp[c] * Gm[(c + r) * r2 + a] : dp[c - r] * Gm[(c - r) * r2 + a]);
        g2 += mac * mca;
      }
    const double ny = sqrt(red[0][0]), nr = sqrt(red[1][0]);
    const double den = 2.0 * sqrt(fmax(a2, 0.0)) * ny + sqrt(fmax(g2, 0.0));
    delta[p] = den > 0.0 ? sqrt(2.0) * nr / den : 0.0;
    if (nrm) {
      nrm[2 * p] = ny;
      nrm[2 * p + 1] = nr;
    }
  }
}

// out (cols x rows) = in^T (rows x cols), both row-major, 32 x 32 tiles through LDS
__global__ void k_transpose(const double* __restrict__ in, long rows, long cols,
                            double* __restrict__ out, long ldo) {
  __shared__ double tile[32][33];
  const long r0 = (long)blockIdx.y * 32, c0 = (long)blockIdx.x * 32;
  for (int k = threadIdx.y; k < 32; k += 8) {
    const long rr = r0 + k, cc = c0 + threadIdx.x;
    tile[k][threadIdx.x] = (rr < rows && cc < cols) ? in[rr * cols + cc] : 0.0;
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += 8) {
    const long cc = c0 + k, rr = r0 + threadIdx.x;
    if (cc < cols && rr < rows) out[cc * ldo + rr] = tile[threadIdx.x][k];
  }
}

// out[i] = sum over s < ns of part[s * stride + i]
__global__ void k_sum_slices(const double* __restrict__ part, int ns, long stride,
                             double* __restrict__ out) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < stride;
       i += (long)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int s = 0; s < ns; ++s) v += part[s * stride + i];
    out[i] = v;
  }
}

// Backward errors from the p-independent operators: one workgroup per
// parameter, ||L Y||^2 = sum of squares of its row of LY = W KT and
// ||Y||^2 = <w, Mq w> with MW = W Mq.
__global__ void __launch_bounds__(NT)
k_ek_delta_ops(const double* __restrict__ LY, long ldly, long ncols, const double* __restrict__ Wp,
               const double* __restrict__ MW, long ldw, int rN, const double* __restrict__ d, int r,
               const double* __restrict__ cst, double* __restrict__ delta, double* __restrict__ nrm) {
  const int p = blockIdx.x;
  double sr = 0.0, sy = 0.0;
  const double* ly = LY + (long)p * ldly;
  for (long c = threadIdx.x; c < ncols; c += NT) sr += ly[c] * ly[c];
  const double* w = Wp + (long)p * ldw;
  const double* mw = MW + (long)p * ldw;
  for (int u = threadIdx.x; u < rN; u += NT) sy += w[u] * mw[u];
  __shared__ double red[2][NT];
  red[0][threadIdx.x] = sy;
  red[1][threadIdx.x] = sr;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double* dp = d + (long)p * r;
    const double* H = cst + 1;
    const double* av = H + r * r;
    const double* Gm = av + r;
    double a2 = cst[0];
    for (int i = 0; i < r; ++i) {
      a2 -= 2.0 * av[i] * dp[i];
      for (int j = 0; j < r; ++j) a2 += dp[i] * dp[j] * H[i * r + j];
    }
    const int r2 = 2 * r;
    double g2 = 0.0;
    for (int a = 0; a < r2; ++a)
      for (int c = 0; c < r2; ++c) {
        const double mac = (a < r ? dp[a] * Gm[(a + r) * r2 + c] : dp[a - r] * Gm[(a - r) * r2 + c]);
        const double mca = (c < r ? dp[c] * Gm[(c + r) * r2 + a] : dp[c - r] * Gm[(c - r) * r2 + a]);
        g2 += mac * mca;
      }
    const double ny = sqrt(fmax(red[0][0], 0.0)), nr = sqrt(red[1][0]);
    const double den = 2.0 * sqrt(fmax(a2, 0.0)) * ny + sqrt(fmax(g2, 0.0));
    delta[p] = den > 0.0 ? sqrt(2.0) * nr / den : 0.0;
    if (nrm) {
      nrm[2 * p] = ny;
      nrm[2 * p + 1] = nr;
    }
  }
}

}  // namespace
}  // namespace lyap

using namespace lyap;

// One level of the projection: the projected seed, the real Schur data of
// T_m for the backward error, and an engine for the projected solves.  A
// level depends on the basis only, so it is kept for later sweeps.
struct EkLevel {
  int m = 0, dim = 0, q = 0;
  lyap_seed_opts opts{};
  lyap_seed_s* proj = nullptr;
  DevBuf Ts, Tst, Zd, Fl, Lz;
  // p-independent operators of the backward error (when they fit): with
  // Ys_u the Schur-basis solution for the unit W = e_b e_k^T (u = b N + k),
  // KT (rNp x ld q) holds (L Z) Ys_u by rows and Mq (rNp x rNp) their Gram
  // matrix, so L Y = W KT and ||Y||^2 = w^T Mq w for every parameter.
  bool ops = false;
  long rNp = 0, colsK = 0;
  DevBuf KT, Mq;
  lyap_engine_s* eng = nullptr;
  DevBuf sol;
  ~EkLevel() {
    if (eng) engine_batch_destroy(eng);
    delete proj;
  }
};

struct lyap_ek_s {
  int64_t n = 0, r = 0;
  int E_diag = 1;
  std::vector<double> A0;       // row-major n x n
  std::vector<double> LU;       // column-major LU factors of A0 (dgetrf)
  std::vector<int> piv;
  std::vector<double> U, V;     // row-major n x r
  std::vector<double> X0V;      // row-major n x r
  std::vector<double> E;        // n (diagonal) or symmetrised n x n row-major
  double t0 = 0.0;
  // basis columns, each contiguous (column-major n x D), A0 and E times them
  std::vector<double> Q, AQ, EQ;
  std::vector<int> bstart{0};   // block b holds columns [bstart[b], bstart[b+1])
  std::vector<int> bplus;       // leading columns of block b from positive powers
  bool exhausted = false;
  // projections onto all D columns built so far, row-major with stride D:
  // TQ = Q^T A0 Q, EM = Q^T E Q (D x D); UQ = Q^T U, VQ = Q^T V, XQ = Q^T X0 V (D x r)
  int D = 0;
  std::vector<double> TQ, EM, UQ, VQ, XQ;
  // p-independent tables of the backward error
  std::vector<double> cst;      // [||A0||_F^2, (U^T U) o (V^T V), diag(U^T A0 V), Gram(P)]
  DevBuf cstd;
  std::vector<std::unique_ptr<EkLevel>> levels;  // index m (0 unused)
  EkLevel* cur = nullptr;
  DevBuf Wbuf, Wp, Gs, Xs, ddev, dl;
  hipStream_t st = nullptr;
  double basis_seconds = 0.0, level_seconds = 0.0;
  double solve_seconds = 0.0, delta_seconds = 0.0;  // projected solves / backward errors
  int64_t batches = 0;

  int nblocks() const { return (int)bstart.size() - 1; }
  const double* col(int j) const { return Q.data() + (size_t)j * n; }
};

namespace {

double dotn(const double* a, const double* b, long n) {
  double s = 0.0;
  for (long i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

void ek_matvec_block(const lyap_ek_s* ek, const double* X, int c, double* Y) {
  // Y (n x c column-major) = A0 X
  const long n = ek->n;
  for (long i = 0; i < n; ++i) {
    const double* Ai = ek->A0.data() + (size_t)i * n;
    for (int k = 0; k < c; ++k) Y[(size_t)k * n + i] = dotn(Ai, X + (size_t)k * n, n);
  }
}

void ek_solve_block(const lyap_ek_s* ek, double* X, int c) {
  if (c == 0) return;
  const int N = (int)ek->n, nrhs = c;
  int info = 0;
  lapack().dgetrs("N", &N, &nrhs, ek->LU.data(), &N, ek->piv.data(), X, &N, &info);
  LYAP_REQUIRE(info == 0, LYAP_E_UNSTABLE, "dgetrs with A0 failed");
}

// Extend the projections TQ, EM, UQ, VQ, XQ to the columns D .. D' - 1.
void ek_project_new(lyap_ek_s* ek) {
  const long n = ek->n, r = ek->r;
  const int D0 = ek->D, D1 = (int)(ek->Q.size() / n);
  if (D1 == D0) return;
  std::vector<double> T1((size_t)D1 * D1), E1((size_t)D1 * D1);
  for (int a = 0; a < D0; ++a)
    for (int b = 0; b < D0; ++b) {
      T1[(size_t)a * D1 + b] = ek->TQ[(size_t)a * D0 + b];
      E1[(size_t)a * D1 + b] = ek->EM[(size_t)a * D0 + b];
    }
  for (int a = 0; a < D1; ++a)
    for (int b = 0; b < D1; ++b) {
      if (a < D0 && b < D0) continue;
      T1[(size_t)a * D1 + b] = dotn(ek->col(a), ek->AQ.data() + (size_t)b * n, n);
      if (b >= a) {
        const double e = dotn(ek->col(a), ek->EQ.data() + (size_t)b * n, n);
        E1[(size_t)a * D1 + b] = e;
        E1[(size_t)b * D1 + a] = e;
      }
    }
  ek->TQ.swap(T1);
  ek->EM.swap(E1);
  ek->UQ.resize((size_t)D1 * r);
  ek->VQ.resize((size_t)D1 * r);
  ek->XQ.resize((size_t)D1 * r);
  for (int a = D0; a < D1; ++a) {
    const double* qa = ek->col(a);
    for (long c = 0; c < r; ++c) {
      double su = 0, sv = 0, sx = 0;
      for (long i = 0; i < n; ++i) {
        su += qa[i] * ek->U[(size_t)i * r + c];
        sv += qa[i] * ek->V[(size_t)i * r + c];
        sx += qa[i] * ek->X0V[(size_t)i * r + c];
      }
      ek->UQ[(size_t)a * r + c] = su;
      ek->VQ[(size_t)a * r + c] = sv;
      ek->XQ[(size_t)a * r + c] = sx;
    }
  }
  ek->D = D1;
}

// Orthogonalise the c candidate columns against the basis (twice) and among
// themselves; append survivors.  Returns the indices that survived.
std::vector<int> ek_append_block(lyap_ek_s* ek, std::vector<double>& W, int c) {
  const long n = ek->n;
  const int dim = (int)(ek->Q.size() / n);
  std::vector<double> nrm0(c);
  for (int k = 0; k < c; ++k) {
    const double* w = W.data() + (size_t)k * n;
    nrm0[k] = std::sqrt(dotn(w, w, n));
  }
  std::vector<double> coef(dim);
  for (int pass = 0; pass < 2 && dim > 0; ++pass)
    for (int k = 0; k < c; ++k) {
      double* w = W.data() + (size_t)k * n;
      for (int j = 0; j < dim; ++j) coef[j] = dotn(ek->col(j), w, n);
      for (int j = 0; j < dim; ++j) {
        const double* qj = ek->col(j);
        const double cj = coef[j];
        for (long i = 0; i < n; ++i) w[i] -= cj * qj[i];
      }
    }
  std::vector<int> kept;
  std::vector<double> newcols;
  newcols.reserve((size_t)c * n);
  for (int k = 0; k < c; ++k) {
    std::vector<double> w(W.begin() + (size_t)k * n, W.begin() + (size_t)(k + 1) * n);
    for (int pass = 0; pass < 2; ++pass)
      for (size_t t = 0; t < kept.size(); ++t) {
        const double* qt = newcols.data() + t * n;
        const double s = dotn(qt, w.data(), n);
        for (long i = 0; i < n; ++i) w[i] -= s * qt[i];
      }
    const double s = std::sqrt(dotn(w.data(), w.data(), n));
    if (s > kDeflate * nrm0[k]) {
      for (long i = 0; i < n; ++i) newcols.push_back(w[i] / s);
      kept.push_back(k);
    }
  }
  const int add = (int)kept.size();
  ek->Q.insert(ek->Q.end(), newcols.begin(), newcols.end());
  std::vector<double> AQn((size_t)add * n), EQn((size_t)add * n);
  if (add) ek_matvec_block(ek, newcols.data(), add, AQn.data());
  for (int k = 0; k < add; ++k) {
    const double* qk = newcols.data() + (size_t)k * n;
    double* out = EQn.data() + (size_t)k * n;
    if (ek->E_diag) {
      for (long i = 0; i < n; ++i) out[i] = ek->E[i] * qk[i];
    } else {
      for (long i = 0; i < n; ++i) out[i] = dotn(ek->E.data() + (size_t)i * n, qk, n);
    }
  }
  ek->AQ.insert(ek->AQ.end(), AQn.begin(), AQn.end());
  ek->EQ.insert(ek->EQ.end(), EQn.begin(), EQn.end());
  ek->bstart.push_back(dim + add);
  ek_project_new(ek);
  return kept;
}

void ek_first_block(lyap_ek_s* ek) {
  const long n = ek->n, r = ek->r, k2 = 2 * r;
  std::vector<double> W((size_t)2 * k2 * n);
  for (long i = 0; i < n; ++i)
    for (long a = 0; a < r; ++a) {
      W[(size_t)a * n + i] = ek->X0V[(size_t)i * r + a];
      W[(size_t)(r + a) * n + i] = ek->U[(size_t)i * r + a];
    }
  std::memcpy(W.data() + (size_t)k2 * n, W.data(), sizeof(double) * k2 * n);
  ek_solve_block(ek, W.data() + (size_t)k2 * n, (int)k2);
  const auto kept = ek_append_block(ek, W, (int)(2 * k2));
  int plus = 0;
  for (int k : kept) plus += k < k2;
  ek->bplus.push_back(plus);
  if (kept.empty()) ek->exhausted = true;
}

// Append the next block: [A0 W+, A0^-1 W-] of the last block.
bool ek_expand(lyap_ek_s* ek) {
  if (ek->exhausted) return false;
  const long n = ek->n;
  const int b = ek->nblocks() - 1;
  const int c0 = ek->bstart[b], c1 = ek->bstart[b + 1], npl = ek->bplus[b];
  const int c = c1 - c0;
  std::vector<double> W((size_t)c * n);
  if (npl) std::memcpy(W.data(), ek->AQ.data() + (size_t)c0 * n, sizeof(double) * npl * n);
  std::memcpy(W.data() + (size_t)npl * n, ek->col(c0 + npl), sizeof(double) * (c - npl) * n);
  ek_solve_block(ek, W.data() + (size_t)npl * n, c - npl);
  const auto kept = ek_append_block(ek, W, c);
  int plus = 0;
  for (int k : kept) plus += k < npl;
  ek->bplus.push_back(plus);
  if (kept.empty()) ek->exhausted = true;
  return !kept.empty();
}

lyap_ek_s* ek_create_impl(int64_t n, int64_t r, const double* A0, const double* U, const double* V,
                          const double* X0V, double t0, const double* E, int E_diag,
                          hipStream_t st) {
  LYAP_REQUIRE(n >= 2 && n <= 65536, LYAP_E_INVAL, "n out of range [2, 65536]");
  LYAP_REQUIRE(r >= 1 && r <= kMaxRank && 4 * r <= n, LYAP_E_INVAL, "r out of range");
  LYAP_REQUIRE(A0 && U && V && X0V && E, LYAP_E_INVAL, "NULL input");
  LYAP_REQUIRE(std::isfinite(t0), LYAP_E_INVAL, "t0 is not finite");
  const LapackFns& L = lapack();
  LYAP_REQUIRE(L.dgetrf && L.dgetrs, LYAP_E_UNSUPPORTED, "no host LAPACK (dgetrf_/dgetrs_)");
  auto t_start = std::chrono::steady_clock::now();
  auto ek = std::make_unique<lyap_ek_s>();
  ek->n = n;
  ek->r = r;
  ek->E_diag = E_diag;
  ek->t0 = t0;
  ek->st = st;
  ek->A0.assign(A0, A0 + (size_t)n * n);
  ek->U.assign(U, U + (size_t)n * r);
  ek->V.assign(V, V + (size_t)n * r);
  ek->X0V.assign(X0V, X0V + (size_t)n * r);
  for (double v : ek->A0) LYAP_REQUIRE(std::isfinite(v), LYAP_E_INVAL, "A0 is not finite");
  for (size_t i = 0; i < ek->U.size(); ++i)
    LYAP_REQUIRE(std::isfinite(ek->U[i]) && std::isfinite(ek->V[i]) && std::isfinite(ek->X0V[i]),
                 LYAP_E_INVAL, "U, V or X0 V is not finite");
  if (E_diag) {
    ek->E.assign(E, E + n);
  } else {
    ek->E.resize((size_t)n * n);
    for (long i = 0; i < n; ++i)
      for (long j = 0; j < n; ++j)
        ek->E[(size_t)i * n + j] = 0.5 * (E[(size_t)i * n + j] + E[(size_t)j * n + i]);
  }
  for (double v : ek->E) LYAP_REQUIRE(std::isfinite(v), LYAP_E_INVAL, "E is not finite");
  // LU of A0 (column-major copy)
  ek->LU.resize((size_t)n * n);
  for (long i = 0; i < n; ++i)
    for (long j = 0; j < n; ++j) ek->LU[(size_t)j * n + i] = A0[(size_t)i * n + j];
  ek->piv.resize(n);
  {
    const int N = (int)n;
    int info = 0;
    L.dgetrf(&N, &N, ek->LU.data(), &N, ek->piv.data(), &info);
    LYAP_REQUIRE(info == 0, LYAP_E_UNSTABLE, "A0 is singular (dgetrf)");
  }
  // tables of the backward error
  {
    std::vector<double>& c = ek->cst;
    c.assign(1 + r * r + r + 4 * r * r, 0.0);
    double a2 = 0.0;
    for (double v : ek->A0) a2 += v * v;
    c[0] = a2;
    std::vector<double> Uc((size_t)r * n), Vc((size_t)r * n), Xc((size_t)r * n);
    for (long i = 0; i < n; ++i)
      for (long a = 0; a < r; ++a) {
        Uc[(size_t)a * n + i] = U[(size_t)i * r + a];
        Vc[(size_t)a * n + i] = V[(size_t)i * r + a];
        Xc[(size_t)a * n + i] = X0V[(size_t)i * r + a];
      }
    for (long a = 0; a < r; ++a)
      for (long b = 0; b < r; ++b)
        c[1 + a * r + b] = dotn(&Uc[(size_t)a * n], &Uc[(size_t)b * n], n) *
                           dotn(&Vc[(size_t)a * n], &Vc[(size_t)b * n], n);
    std::vector<double> AV((size_t)r * n);
    ek_matvec_block(ek.get(), Vc.data(), (int)r, AV.data());
    for (long a = 0; a < r; ++a) c[1 + r * r + a] = dotn(&Uc[(size_t)a * n], &AV[(size_t)a * n], n);
    // Gram of P = [X0 V, U]
    const long r2 = 2 * r;
    double* G = c.data() + 1 + r * r + r;
    auto pcol = [&](long a) { return a < r ? &Xc[(size_t)a * n] : &Uc[(size_t)(a - r) * n]; };
    for (long a = 0; a < r2; ++a)
      for (long b = 0; b < r2; ++b) G[a * r2 + b] = dotn(pcol(a), pcol(b), n);
    ek->cstd.alloc(c.size() * sizeof(double));
    LYAP_HIP(hipMemcpyAsync(ek->cstd.p, c.data(), ek->cstd.bytes, hipMemcpyHostToDevice, st));
    LYAP_HIP(hipStreamSynchronize(st));
  }
  ek_first_block(ek.get());
  LYAP_REQUIRE(!ek->exhausted, LYAP_E_INVAL, "P = [X0 V, U] is zero");
  ek->basis_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return ek.release();
}

bool same_opts(const lyap_seed_opts& a, const lyap_seed_opts& b) {
  return a.basis == b.basis && a.max_eig_cond == b.max_eig_cond && a.tsvd_rank == b.tsvd_rank;
}

// The backward-error operators of a level (see EkLevel).  One batched
// quasi-triangular solve over the r N unit right-hand sides, then two GEMMs.
void ek_build_ops(lyap_ek_s* ek, EkLevel* lv, const std::vector<double>& Flh,
                  const std::vector<double>& Zh, const std::vector<double>& Lzh) {
  const long r = ek->r, N = lv->dim, ld = lv->proj->ld, q = lv->q;
  const long rN = r * N, rNp = pad_to(rN, 128), l2 = ld * ld;
  const size_t ybytes = (size_t)rN * l2 * sizeof(double);
  if (q == 0 || 2 * ybytes > kOpBytes) return;  // invariant level, or too large: direct route
  hipStream_t st = ek->st;
  // per-problem factors: F row u = Fl row (u / N), G row u = Z row (u % N)
  std::vector<double> Fr((size_t)rN * ld, 0.0), Gr((size_t)rN * ld, 0.0);
  for (long u = 0; u < rN; ++u) {
    const long b = u / N, k = u % N;
    std::memcpy(&Fr[(size_t)u * ld], &Flh[(size_t)b * ld], sizeof(double) * ld);
    for (long j = 0; j < N; ++j) Gr[(size_t)u * ld + j] = Zh[(size_t)k * N + j];
  }
  DevBuf Frd(Fr.size() * sizeof(double)), Grd(Gr.size() * sizeof(double)), Yu(ybytes);
  LYAP_HIP(hipMemcpyAsync(Frd.p, Fr.data(), Frd.bytes, hipMemcpyHostToDevice, st));
  LYAP_HIP(hipMemcpyAsync(Grd.p, Gr.data(), Grd.bytes, hipMemcpyHostToDevice, st));
  LYAP_HIP(hipMemsetAsync(Yu.p, 0, ybytes, st));
  trilyap_launch(lv->Ts.as<double>(), lv->Tst.as<double>(), Yu.as<double>(), l2, nullptr, 0,
                 Frd.as<double>(), Grd.as<double>(), ld, 1, (int)N, (int)ld, (int)rN, nullptr,
                 nullptr, st, ld);
  // KT: rows (u, j) of Yu (column j of Ys_u) times (L Z)^T, q columns stored
  std::vector<double> LzT((size_t)ld * 128, 0.0);
  for (long a = 0; a < q; ++a)
    for (long i = 0; i < N; ++i) LzT[(size_t)i * 128 + a] = Lzh[(size_t)a * ld + i];
  DevBuf LzTd(LzT.size() * sizeof(double));
  LYAP_HIP(hipMemcpyAsync(LzTd.p, LzT.data(), LzTd.bytes, hipMemcpyHostToDevice, st));
  lv->colsK = ld * q;
  lv->rNp = rNp;
  lv->KT.alloc((size_t)rNp * lv->colsK * sizeof(double));
  LYAP_HIP(hipMemsetAsync(lv->KT.p, 0, lv->KT.bytes, st));
  gemm64_rm(Yu.as<double>(), ld, LzTd.as<double>(), 128, lv->KT.as<double>(), q, rN * ld, 128, ld,
            q, st);
  // Mq = Yflat Yflat^T with Yflat (rN x ld^2): through the transpose
  {
    DevBuf YT((size_t)l2 * rNp * sizeof(double));
    LYAP_HIP(hipMemsetAsync(YT.p, 0, YT.bytes, st));
    dim3 grid((unsigned)((l2 + 31) / 32), (unsigned)((rN + 31) / 32));
    hipLaunchKernelGGL(k_transpose, grid, dim3(32, 8), 0, st, Yu.as<double>(), rN, l2,
                       YT.as<double>(), rNp);
    LYAP_HIP(hipGetLastError());
    // K = ld^2 is long and the output has few tiles: 16 K-slices, summed after
    constexpr int kSlices = 16;
    const long kc = l2 / kSlices;  // ld is a multiple of 128, so kc is a multiple of the K tile
    const size_t pe = (size_t)rNp * rNp;
    DevBuf part(kSlices * pe * sizeof(double));
    LYAP_HIP(hipMemsetAsync(part.p, 0, part.bytes, st));
    for (int c = 0; c < kSlices; ++c)
      gemm64_rm(Yu.as<double>() + c * kc, l2, YT.as<double>() + (size_t)c * kc * rNp, rNp,
                part.as<double>() + c * pe, rNp, rN, rNp, kc, rNp, st);
    lv->Mq.alloc(pe * sizeof(double));
    hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)std::min<size_t>((pe + 255) / 256, 65535)),
                       dim3(256), 0, st, part.as<double>(), kSlices, (long)pe, lv->Mq.as<double>());
    LYAP_HIP(hipGetLastError());
    LYAP_HIP(hipStreamSynchronize(st));
  }
  lv->ops = true;
}

// Level m (blocks 0..m-1): the projected seed and the backward-error data.
EkLevel* ek_build_level(lyap_ek_s* ek, int mm, const lyap_seed_opts& o) {
  const long r = ek->r;
  const int N = ek->bstart[mm];
  LYAP_REQUIRE(N >= r, LYAP_E_INVAL, "projected dimension below the rank");
  const int q = mm < ek->nblocks() ? ek->bstart[mm + 1] - ek->bstart[mm] : 0;
  const int D = ek->D;
  auto lv = std::make_unique<EkLevel>();
  lv->m = mm;
  lv->dim = N;
  lv->q = q;
  lv->opts = o;
  std::vector<double> T((size_t)N * N), Em((size_t)N * N), Um((size_t)N * r), Vm((size_t)N * r),
      Ct((size_t)r * N);
  for (int a = 0; a < N; ++a) {
    for (int b = 0; b < N; ++b) {
      T[(size_t)a * N + b] = ek->TQ[(size_t)a * D + b];
      Em[(size_t)a * N + b] = ek->EM[(size_t)a * D + b];
    }
    for (long c = 0; c < r; ++c) {
      Um[(size_t)a * r + c] = ek->UQ[(size_t)a * r + c];
      Vm[(size_t)a * r + c] = ek->VQ[(size_t)a * r + c];
      Ct[(size_t)c * N + a] = ek->XQ[(size_t)a * r + c];
    }
  }
  ProjRhs pr{Ct.data(), ek->t0};
  lv->proj = factor_projected(N, r, T.data(), Um.data(), Vm.data(), Em.data(), pr, &o, ek->st);
  // real Schur form of T_m for the backward error
  std::vector<double> Th((size_t)N * N), Zh((size_t)N * N);
  LYAP_REQUIRE(real_schur(N, T.data(), Th.data(), Zh.data(), nullptr), LYAP_E_UNSTABLE,
               "real Schur iteration on T_m did not converge");
  const long ld = lv->proj->ld;
  const size_t mat = (size_t)ld * ld * sizeof(double);
  std::vector<double> Tp((size_t)ld * ld, 0.0), Ttp((size_t)ld * ld, 0.0), Zp((size_t)ld * ld, 0.0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      Tp[(size_t)i * ld + j] = Th[(size_t)i * N + j];
      Ttp[(size_t)j * ld + i] = Th[(size_t)i * N + j];
      Zp[(size_t)i * ld + j] = Zh[(size_t)i * N + j];
    }
  // Fl = U_m^T Z (r x ld); Lz = L Z (q x ld), L = rows N..N+q-1 of Q^T A0 Q, columns < N
  std::vector<double> Flh((size_t)r * ld, 0.0), Lzh((size_t)std::max(q, 1) * ld, 0.0);
  for (long a = 0; a < r; ++a)
    for (int j = 0; j < N; ++j) {
      double s = 0.0;
      for (int i = 0; i < N; ++i) s += Um[(size_t)i * r + a] * Zh[(size_t)i * N + j];
      Flh[(size_t)a * ld + j] = s;
    }
  for (int a = 0; a < q; ++a)
    for (int j = 0; j < N; ++j) {
      double s = 0.0;
      for (int i = 0; i < N; ++i) s += ek->TQ[(size_t)(N + a) * D + i] * Zh[(size_t)i * N + j];
      Lzh[(size_t)a * ld + j] = s;
    }
  hipStream_t st = ek->st;
  lv->Ts.alloc(mat);
  lv->Tst.alloc(mat);
  lv->Zd.alloc(mat);
  lv->Fl.alloc(Flh.size() * sizeof(double));
  lv->Lz.alloc(Lzh.size() * sizeof(double));
  LYAP_HIP(hipMemcpyAsync(lv->Ts.p, Tp.data(), mat, hipMemcpyHostToDevice, st));
  LYAP_HIP(hipMemcpyAsync(lv->Tst.p, Ttp.data(), mat, hipMemcpyHostToDevice, st));
  LYAP_HIP(hipMemcpyAsync(lv->Zd.p, Zp.data(), mat, hipMemcpyHostToDevice, st));
  LYAP_HIP(hipMemcpyAsync(lv->Fl.p, Flh.data(), lv->Fl.bytes, hipMemcpyHostToDevice, st));
  LYAP_HIP(hipMemcpyAsync(lv->Lz.p, Lzh.data(), lv->Lz.bytes, hipMemcpyHostToDevice, st));
  LYAP_HIP(hipStreamSynchronize(st));
  ek_build_ops(ek, lv.get(), Flh, Zh, Lzh);
  return lv.release();
}

// Make level m current (built on first use, kept afterwards).
EkLevel* ek_level(lyap_ek_s* ek, int m, const lyap_seed_opts* popts) {
  LYAP_REQUIRE(m >= 1 && m <= 100000, LYAP_E_INVAL, "level out of range");
  lyap_seed_opts o{};
  o.basis = popts ? popts->basis : LYAP_BASIS_AUTO;
  o.E_is_diag = 0;
  o.max_eig_cond = popts ? popts->max_eig_cond : 0.0;
  o.tsvd_rank = popts ? popts->tsvd_rank : 0;
  auto t0 = std::chrono::steady_clock::now();
  while (ek->nblocks() < m + 1 && !ek->exhausted) ek_expand(ek);
  auto t1 = std::chrono::steady_clock::now();
  ek->basis_seconds += std::chrono::duration<double>(t1 - t0).count();
  const int mm = std::min(m, ek->nblocks());
  if ((int)ek->levels.size() <= mm) ek->levels.resize(mm + 1);
  auto& slot = ek->levels[mm];
  if (!slot || !same_opts(slot->opts, o)) {
    slot.reset();
    slot.reset(ek_build_level(ek, mm, o));
    ek->level_seconds +=
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
  }
  ek->cur = slot.get();
  return ek->cur;
}

// Backward errors of P parameters at level lv from W (P x r x dim).
void ek_delta_impl(lyap_ek_s* ek, EkLevel* lv, int64_t P, const double* d_dev, const double* W_dev,
                   double* delta_dev, double* nrm_dev) {
  const long r = ek->r, N = lv->dim, ld = lv->proj->ld;
  hipStream_t st = ek->st;
  if (lv->ops) {
    const long rN = r * N, rNp = lv->rNp, cols = lv->colsK;
    const size_t wb = (size_t)P * rNp * sizeof(double);
    if (ek->Wp.bytes < wb) ek->Wp.alloc(wb);
    if (ek->Gs.bytes < wb) ek->Gs.alloc(wb);
    const size_t lb = (size_t)P * cols * sizeof(double);
    if (ek->Xs.bytes < lb) ek->Xs.alloc(lb);
    LYAP_HIP(hipMemsetAsync(ek->Wp.p, 0, wb, st));
    const int ub = (int)std::min<long>((rN + 255) / 256, 64);
    hipLaunchKernelGGL(k_pad_rows_ek, dim3(ub, (unsigned)P), dim3(256), 0, st, ek->Wp.as<double>(),
                       rNp, W_dev, rN, (int)rN);
    LYAP_HIP(hipGetLastError());
    gemm64_rm(ek->Wp.as<double>(), rNp, lv->KT.as<double>(), cols, ek->Xs.as<double>(), cols,
              (long)P, cols, rNp, cols, st);
    gemm64_rm(ek->Wp.as<double>(), rNp, lv->Mq.as<double>(), rNp, ek->Gs.as<double>(), rNp, (long)P,
              rNp, rNp, rNp, st);
    hipLaunchKernelGGL(k_ek_delta_ops, dim3((unsigned)P), dim3(NT), 0, st, ek->Xs.as<double>(), cols,
                       cols, ek->Wp.as<double>(), ek->Gs.as<double>(), rNp, (int)rN, d_dev, (int)r,
                       ek->cstd.as<double>(), delta_dev, nrm_dev);
    LYAP_HIP(hipGetLastError());
    return;
  }
  for (int64_t p0 = 0; p0 < P; p0 += kDeltaChunk) {
    const int cnt = (int)std::min<int64_t>(kDeltaChunk, P - p0);
    const size_t rowsb = (size_t)cnt * r * ld * sizeof(double);
    if (ek->Wp.bytes < rowsb) ek->Wp.alloc(rowsb);
    if (ek->Gs.bytes < rowsb) ek->Gs.alloc(rowsb);
    const size_t xb = (size_t)cnt * ld * ld * sizeof(double);
    if (ek->Xs.bytes < xb) ek->Xs.alloc(xb);
    LYAP_HIP(hipMemsetAsync(ek->Wp.p, 0, rowsb, st));
    LYAP_HIP(hipMemsetAsync(ek->Gs.p, 0, rowsb, st));
    const int ub = (int)std::min<long>((N + 255) / 256, 64);
    hipLaunchKernelGGL(k_pad_rows_ek, dim3(ub, cnt * r), dim3(256), 0, st, ek->Wp.as<double>(), ld,
                       W_dev + (size_t)p0 * r * N, N, (int)N);
    LYAP_HIP(hipGetLastError());
    // Gs = W Z: the per-parameter factor of Z^T (U_m W + W^T U_m^T) Z
    gemm64_rm(ek->Wp.as<double>(), ld, lv->Zd.as<double>(), ld, ek->Gs.as<double>(), ld,
              (long)cnt * r, ld, ld, ld, st);
    trilyap_launch(lv->Ts.as<double>(), lv->Tst.as<double>(), ek->Xs.as<double>(), ld * ld, nullptr,
                   0, lv->Fl.as<double>(), ek->Gs.as<double>(), r * ld, (int)r, (int)N, (int)ld,
                   cnt, nullptr, nullptr, st);
    hipLaunchKernelGGL(k_ek_delta, dim3(cnt), dim3(NT), 0, st, ek->Xs.as<double>(), ld * ld, (int)N,
                       (int)ld, lv->Lz.as<double>(), lv->q, d_dev + (size_t)p0 * r, (int)r,
                       ek->cstd.as<double>(), delta_dev + p0, nrm_dev ? nrm_dev + 2 * p0 : nullptr);
    LYAP_HIP(hipGetLastError());
  }
}

// Projected solves of P parameters at level lv, then their backward errors.
void ek_solve_level(lyap_ek_s* ek, EkLevel* lv, int64_t P, const double* d_dev,
                    const lyap_solve_opts* opts, double* W_dev, double* delta_dev, double* nrm_dev,
                    lyap_result* res) {
  LYAP_REQUIRE(P >= 1 && d_dev && W_dev && delta_dev && res, LYAP_E_INVAL, "bad argument");
  if (!lv->eng || !engine_batch_fits(lv->eng, P, opts)) {
    if (lv->eng) engine_batch_destroy(lv->eng);
    lv->eng = nullptr;
    const long long cap = std::max<long long>(P, 64);
    lv->sol.alloc((size_t)cap * ek->r * lv->proj->ld * sizeof(double));
    lv->eng = engine_batch_create(lv->proj, cap, opts, ek->st, lv->sol.as<double>());
  } else {
    engine_batch_reset(lv->eng, ek->st);
  }
  auto t0 = std::chrono::steady_clock::now();
  engine_batch_run(lv->eng, P, d_dev, W_dev, res);
  auto t1 = std::chrono::steady_clock::now();
  ek_delta_impl(ek, lv, P, d_dev, W_dev, delta_dev, nrm_dev);
  LYAP_HIP(hipStreamSynchronize(ek->st));
  ek->solve_seconds += std::chrono::duration<double>(t1 - t0).count();
  ek->delta_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
  ++ek->batches;
}

// Algorithm EKSM_opt: parameters in order; at each level the queue is tested
// from its head and the longest accepted prefix leaves; the first failure
// moves every remaining parameter to the next level.  The queue head is
// solved in chunks that grow fourfold after every fully accepted chunk
// (1, 4, 16, ...) and restart at one on a new level, so the accepted prefix is
// the one the sequential loop finds while the solves stay batched.
void ek_sweep_impl(lyap_ek_s* ek, int64_t P, const double* d_host, const lyap_solve_opts* opts,
                   const lyap_seed_opts* popts, double eps, int m_start, int m_max,
                   int check_every, lyap_ek_result* out) {
  const long r = ek->r;
  for (int64_t i = 0; i < P * r; ++i)
    LYAP_REQUIRE(std::isfinite(d_host[i]), LYAP_E_INVAL, "non-finite parameter");
  for (int64_t i = 0; i < P; ++i) out[i] = lyap_ek_result{LYAP_E_NOCONV, 0, 0, 0, NAN, NAN};
  if (ek->ddev.bytes < (size_t)P * r * sizeof(double)) ek->ddev.alloc((size_t)P * r * sizeof(double));
  if (ek->dl.bytes < (size_t)P * sizeof(double)) ek->dl.alloc((size_t)P * sizeof(double));
  LYAP_HIP(hipMemcpyAsync(ek->ddev.p, d_host, (size_t)P * r * sizeof(double), hipMemcpyHostToDevice,
                          ek->st));
  std::vector<double> delta;
  std::vector<lyap_result> res;
  int64_t pos = 0, chunk = 1;
  int m = m_start;
  while (pos < P && m <= m_max) {
    EkLevel* lv = ek_level(ek, m, popts);
    const int64_t cnt = std::min<int64_t>(chunk, P - pos);
    const size_t wb = (size_t)cnt * r * lv->dim * sizeof(double);
    if (ek->Wbuf.bytes < wb) ek->Wbuf.alloc(wb);
    res.resize(cnt);
    ek_solve_level(ek, lv, cnt, ek->ddev.as<double>() + (size_t)pos * r, opts, ek->Wbuf.as<double>(),
                   ek->dl.as<double>() + pos, nullptr, res.data());
    delta.resize(cnt);
    LYAP_HIP(hipMemcpyAsync(delta.data(), ek->dl.as<double>() + pos, (size_t)cnt * sizeof(double),
                            hipMemcpyDeviceToHost, ek->st));
    LYAP_HIP(hipStreamSynchronize(ek->st));
    const bool invariant = lv->q == 0;  // the projection is exact
    int64_t t = 0;
    for (; t < cnt; ++t) {
      lyap_ek_result& o = out[pos + t];
      o.iters += res[t].iters;
      o.level = lv->m;
      o.dim = lv->dim;
      o.delta = delta[t];
      o.trace = res[t].trace;
      if (res[t].status != LYAP_OK) {
        o.status = res[t].status;
        break;
      }
      if (!(delta[t] <= eps || invariant)) break;
      o.status = LYAP_OK;
    }
    // chunk members after the first failure were solved but are not tested at
    // this level (the sequential loop never reaches them): their work counts
    for (int64_t u = t + 1; u < cnt; ++u) out[pos + u].iters += res[u].iters;
    pos += t;
    if (t < cnt) {
      if (invariant) {
        ++pos;  // the space cannot grow: the projected solve itself failed
        chunk = 1;
        continue;
      }
      m = lv->m + check_every;
      chunk = 1;
    } else {
      chunk = std::min<int64_t>(4 * chunk, P);
    }
  }
}

}  // namespace

extern "C" {

lyap_status seed_x0v(lyap_seed sd, double* X0V) {
  if (!sd || !X0V) return LYAP_E_INVAL;
  LYAP_TRY({
    const long r = sd->r, n = sd->n, ld = sd->ld;
    DevBuf out((size_t)r * ld * sizeof(double));
    LYAP_HIP(hipMemsetAsync(out.p, 0, out.bytes, sd->stream));
    // physical V^T X0 = c0 Tout (the map the solutions take back from the basis)
    gemm64_rm(sd->c0.as<double>(), ld, sd->Tout.as<double>(), ld, out.as<double>(), ld, r, ld, ld,
              n, sd->stream);
    std::vector<double> h((size_t)r * ld);
    LYAP_HIP(hipMemcpyAsync(h.data(), out.p, out.bytes, hipMemcpyDeviceToHost, sd->stream));
    LYAP_HIP(hipStreamSynchronize(sd->stream));
    for (long i = 0; i < n; ++i)
      for (long a = 0; a < r; ++a) X0V[(size_t)i * r + a] = h[(size_t)a * ld + i];
  });
  return LYAP_OK;
}

lyap_status ek_create(int64_t n, int64_t r, const double* A0, const double* U, const double* V,
                      const double* X0V, double t0, const double* E, int32_t E_is_diag,
                      void* hip_stream, lyap_ek* out) {
  if (!out) return LYAP_E_INVAL;
  *out = nullptr;
  LYAP_TRY(*out = ek_create_impl(n, r, A0, U, V, X0V, t0, E, E_is_diag, (hipStream_t)hip_stream));
  return LYAP_OK;
}

lyap_status ek_set_level(lyap_ek ek, int32_t m, const lyap_seed_opts* proj_opts) {
  if (!ek) return LYAP_E_INVAL;
  LYAP_TRY(ek_level(ek, m, proj_opts));
  return LYAP_OK;
}

lyap_status ek_solve(lyap_ek ek, int64_t P, const double* d_dev, const lyap_solve_opts* opts,
                     double* W_dev, double* delta_dev, double* norms_dev, lyap_result* res_host) {
  if (!ek) return LYAP_E_INVAL;
  LYAP_TRY({
    LYAP_REQUIRE(ek->cur, LYAP_E_INVAL, "ek_set_level was not called");
    ek_solve_level(ek, ek->cur, P, d_dev, opts, W_dev, delta_dev, norms_dev, res_host);
  });
  return LYAP_OK;
}

lyap_status ek_sweep(lyap_ek ek, int64_t P, const double* d_host, const lyap_solve_opts* opts,
                     const lyap_seed_opts* proj_opts, double eps, int32_t m_start,
                     int32_t m_max, int32_t check_every, lyap_ek_result* out) {
  if (!ek || P < 1 || !d_host || !out || !(eps > 0) || m_start < 1 || m_max < m_start ||
      check_every < 1)
    return LYAP_E_INVAL;
  LYAP_TRY(ek_sweep_impl(ek, P, d_host, opts, proj_opts, eps, m_start, m_max, check_every, out));
  return LYAP_OK;
}

lyap_status ek_info(lyap_ek ek, lyap_ek_info* o) {
  if (!ek || !o) return LYAP_E_INVAL;
  o->n = ek->n;
  o->r = ek->r;
  o->level = ek->cur ? ek->cur->m : 0;
  o->dim = ek->cur ? ek->cur->dim : 0;
  o->blocks = ek->nblocks();
  o->basis_cols = ek->D;
  o->exhausted = ek->exhausted ? 1 : 0;
  o->proj_basis = ek->cur ? ek->cur->proj->basis : -1;
  o->proj_cond = ek->cur ? ek->cur->proj->cond_est : 0.0;
  o->basis_seconds = ek->basis_seconds;
  o->level_seconds = ek->level_seconds;
  o->solve_seconds = ek->solve_seconds;
  o->delta_seconds = ek->delta_seconds;
  o->batches = ek->batches;
  return LYAP_OK;
}

lyap_status ek_release(lyap_ek ek) {
  if (!ek) return LYAP_E_INVAL;
  delete ek;
  return LYAP_OK;
}

}  // extern "C"
