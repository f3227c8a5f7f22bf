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

}  // namespace
}  // namespace lyap

using namespace lyap;

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
  // basis columns, each contiguous (column-major n x dim), and A0 times them
  std::vector<double> Q, AQ;
  std::vector<int> bstart{0};   // block b holds columns [bstart[b], bstart[b+1])
  std::vector<int> bplus;       // leading columns of block b from positive powers
  bool exhausted = false;
  // p-independent tables of the backward error
  std::vector<double> cst;      // [||A0||_F^2, (U^T U) o (V^T V), diag(U^T A0 V), Gram(P)]
  // current level
  int level = 0, dim = 0, q = 0;
  lyap_seed_s* proj = nullptr;
  DevBuf Ts, Tst, Zd, Fl, Lz, cstd;
  DevBuf Wbuf, Wp, Gs, Xs, ddev, dl;
  hipStream_t st = nullptr;
  double basis_seconds = 0.0, level_seconds = 0.0;

  int nblocks() const { return (int)bstart.size() - 1; }
  const double* col(int j) const { return Q.data() + (size_t)j * n; }

  ~lyap_ek_s() { delete proj; }
};

namespace {

void ek_matvec_block(const lyap_ek_s* ek, const double* X, int c, double* Y) {
  // Y (n x c column-major) = A0 X
  const long n = ek->n;
  for (int k = 0; k < c; ++k) std::memset(Y + (size_t)k * n, 0, sizeof(double) * n);
  for (long i = 0; i < n; ++i) {
    const double* Ai = ek->A0.data() + (size_t)i * n;
    for (int k = 0; k < c; ++k) {
      const double* x = X + (size_t)k * n;
      double s = 0.0;
      for (long j = 0; j < n; ++j) s += Ai[j] * x[j];
      Y[(size_t)k * n + i] = s;
    }
  }
}

void ek_solve_block(const lyap_ek_s* ek, double* X, int c) {
  if (c == 0) return;
  const int N = (int)ek->n, nrhs = c;
  int info = 0;
  lapack().dgetrs("N", &N, &nrhs, ek->LU.data(), &N, ek->piv.data(), X, &N, &info);
  LYAP_REQUIRE(info == 0, LYAP_E_UNSTABLE, "dgetrs with A0 failed");
}

// Orthogonalise the c candidate columns against the basis (twice) and among
// themselves; append survivors.  Returns the indices that survived.
std::vector<int> ek_append_block(lyap_ek_s* ek, std::vector<double>& W, int c) {
  const long n = ek->n;
  const int dim = (int)(ek->Q.size() / n);
  std::vector<double> nrm0(c);
  for (int k = 0; k < c; ++k) {
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += W[(size_t)k * n + i] * W[(size_t)k * n + i];
    nrm0[k] = std::sqrt(s);
  }
  std::vector<double> coef(dim);
  for (int pass = 0; pass < 2 && dim > 0; ++pass)
    for (int k = 0; k < c; ++k) {
      double* w = W.data() + (size_t)k * n;
      for (int j = 0; j < dim; ++j) {
        const double* qj = ek->col(j);
        double s = 0.0;
        for (long i = 0; i < n; ++i) s += qj[i] * w[i];
        coef[j] = s;
      }
      for (int j = 0; j < dim; ++j) {
        const double* qj = ek->col(j);
        const double cj = coef[j];
        for (long i = 0; i < n; ++i) w[i] -= cj * qj[i];
      }
    }
  std::vector<int> kept;
  std::vector<const double*> fresh;
  std::vector<double> newcols;
  newcols.reserve((size_t)c * n);
  for (int k = 0; k < c; ++k) {
    std::vector<double> w(W.begin() + (size_t)k * n, W.begin() + (size_t)(k + 1) * n);
    for (int pass = 0; pass < 2; ++pass)
      for (size_t t = 0; t < kept.size(); ++t) {
        const double* qt = newcols.data() + t * n;
        double s = 0.0;
        for (long i = 0; i < n; ++i) s += qt[i] * w[i];
        for (long i = 0; i < n; ++i) w[i] -= s * qt[i];
      }
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += w[i] * w[i];
    s = std::sqrt(s);
    if (s > kDeflate * nrm0[k]) {
      for (long i = 0; i < n; ++i) newcols.push_back(w[i] / s);
      kept.push_back(k);
    }
  }
  const int add = (int)kept.size();
  ek->Q.insert(ek->Q.end(), newcols.begin(), newcols.end());
  std::vector<double> AQn((size_t)add * n);
  if (add) ek_matvec_block(ek, newcols.data(), add, AQn.data());
  ek->AQ.insert(ek->AQ.end(), AQn.begin(), AQn.end());
  ek->bstart.push_back(dim + add);
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

double dotn(const double* a, const double* b, long n) {
  double s = 0.0;
  for (long i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
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
  }
  ek_first_block(ek.get());
  LYAP_REQUIRE(!ek->exhausted, LYAP_E_INVAL, "P = [X0 V, U] is zero");
  ek->basis_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return ek.release();
}

// Projected seed and backward-error data for level m (blocks 0..m-1).
void ek_set_level_impl(lyap_ek_s* ek, int m, const lyap_seed_opts* popts) {
  LYAP_REQUIRE(m >= 1 && m <= 100000, LYAP_E_INVAL, "level out of range");
  auto t_start = std::chrono::steady_clock::now();
  while (ek->nblocks() < m + 1 && !ek->exhausted) ek_expand(ek);
  ek->basis_seconds +=
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  const int mm = std::min(m, ek->nblocks());
  const long n = ek->n, r = ek->r;
  const int N = ek->bstart[mm];
  LYAP_REQUIRE(N >= r, LYAP_E_INVAL, "projected dimension below the rank");
  const int q = mm < ek->nblocks() ? ek->bstart[mm + 1] - ek->bstart[mm] : 0;
  auto t1 = std::chrono::steady_clock::now();
  // T_m, L, U_m, V_m, C, E_m (row-major)
  std::vector<double> T((size_t)N * N), Lc((size_t)std::max(q, 1) * N), Um((size_t)N * r),
      Vm((size_t)N * r), Ct((size_t)r * N), Em((size_t)N * N);
  for (int a = 0; a < N; ++a) {
    const double* qa = ek->col(a);
    for (int b = 0; b < N; ++b) T[(size_t)a * N + b] = dotn(qa, ek->AQ.data() + (size_t)b * n, n);
    for (long c = 0; c < r; ++c) {
      double su = 0, sv = 0, sx = 0;
      for (long i = 0; i < n; ++i) {
        su += qa[i] * ek->U[(size_t)i * r + c];
        sv += qa[i] * ek->V[(size_t)i * r + c];
        sx += qa[i] * ek->X0V[(size_t)i * r + c];
      }
      Um[(size_t)a * r + c] = su;
      Vm[(size_t)a * r + c] = sv;
      Ct[(size_t)c * N + a] = sx;
    }
  }
  for (int a = 0; a < q; ++a) {
    const double* qa = ek->col(N + a);
    for (int b = 0; b < N; ++b) Lc[(size_t)a * N + b] = dotn(qa, ek->AQ.data() + (size_t)b * n, n);
  }
  {
    std::vector<double> EQ((size_t)N * n);  // column b: E q_b
    for (int b = 0; b < N; ++b) {
      const double* qb = ek->col(b);
      double* out = EQ.data() + (size_t)b * n;
      if (ek->E_diag) {
        for (long i = 0; i < n; ++i) out[i] = ek->E[i] * qb[i];
      } else {
        for (long i = 0; i < n; ++i) out[i] = dotn(ek->E.data() + (size_t)i * n, qb, n);
      }
    }
    for (int a = 0; a < N; ++a)
      for (int b = a; b < N; ++b) {
        const double v = dotn(ek->col(a), EQ.data() + (size_t)b * n, n);
        Em[(size_t)a * N + b] = v;
        Em[(size_t)b * N + a] = v;
      }
  }
  // projected seed (replaces the previous level's)
  lyap_seed_opts o{};
  o.basis = popts ? popts->basis : LYAP_BASIS_AUTO;
  o.E_is_diag = 0;
  o.max_eig_cond = popts ? popts->max_eig_cond : 0.0;
  o.tsvd_rank = popts ? popts->tsvd_rank : 0;
  delete ek->proj;
  ek->proj = nullptr;
  ek->level = 0;
  ProjRhs pr{Ct.data(), ek->t0};
  ek->proj = factor_projected(N, r, T.data(), Um.data(), Vm.data(), Em.data(), pr, &o, ek->st);
  // real Schur form of T_m for the backward error
  std::vector<double> Th((size_t)N * N), Zh((size_t)N * N);
  LYAP_REQUIRE(real_schur(N, T.data(), Th.data(), Zh.data(), nullptr), LYAP_E_UNSTABLE,
               "real Schur iteration on T_m did not converge");
  const long ld = ek->proj->ld;
  const size_t mat = (size_t)ld * ld * sizeof(double);
  std::vector<double> Tp((size_t)ld * ld, 0.0), Ttp((size_t)ld * ld, 0.0), Zp((size_t)ld * ld, 0.0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      Tp[(size_t)i * ld + j] = Th[(size_t)i * N + j];
      Ttp[(size_t)j * ld + i] = Th[(size_t)i * N + j];
      Zp[(size_t)i * ld + j] = Zh[(size_t)i * N + j];
    }
  // Fl = U_m^T Z (r x ld), Lz = L Z (q x ld)
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
      for (int i = 0; i < N; ++i) s += Lc[(size_t)a * N + i] * Zh[(size_t)i * N + j];
      Lzh[(size_t)a * ld + j] = s;
    }
  hipStream_t st = ek->st;
  ek->Ts.alloc(mat);
  ek->Tst.alloc(mat);
  ek->Zd.alloc(mat);
  ek->Fl.alloc(Flh.size() * sizeof(double));
  ek->Lz.alloc(Lzh.size() * sizeof(double));
  ek->cstd.alloc(ek->cst.size() * sizeof(double));
  LYAP_HIP(hipMemcpyAsync(ek->Ts.p, Tp.data(), mat, hipMemcpyHostToDevice, st));
  LYAP_HIP(hipMemcpyAsync(ek->Tst.p, Ttp.data(), mat, hipMemcpyHostToDevice, st));
  LYAP_HIP(hipMemcpyAsync(ek->Zd.p, Zp.data(), mat, hipMemcpyHostToDevice, st));
  LYAP_HIP(hipMemcpyAsync(ek->Fl.p, Flh.data(), ek->Fl.bytes, hipMemcpyHostToDevice, st));
  LYAP_HIP(hipMemcpyAsync(ek->Lz.p, Lzh.data(), ek->Lz.bytes, hipMemcpyHostToDevice, st));
  LYAP_HIP(hipMemcpyAsync(ek->cstd.p, ek->cst.data(), ek->cstd.bytes, hipMemcpyHostToDevice, st));
  LYAP_HIP(hipStreamSynchronize(st));
  ek->level = mm;
  ek->dim = N;
  ek->q = q;
  ek->level_seconds +=
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
}

// Backward errors of P parameters at the current level from W (P x r x dim).
void ek_delta_impl(lyap_ek_s* ek, int64_t P, const double* d_dev, const double* W_dev,
                   double* delta_dev, double* nrm_dev) {
  const long r = ek->r, N = ek->dim, ld = ek->proj->ld;
  hipStream_t st = ek->st;
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
    // Gs = W Z: the per-parameter factor of Zs^T (U_m W + W^T U_m^T) Zs
    gemm64_rm(ek->Wp.as<double>(), ld, ek->Zd.as<double>(), ld, ek->Gs.as<double>(), ld,
              (long)cnt * r, ld, ld, ld, st);
    trilyap_launch(ek->Ts.as<double>(), ek->Tst.as<double>(), ek->Xs.as<double>(), ld * ld, nullptr,
                   0, ek->Fl.as<double>(), ek->Gs.as<double>(), r * ld, (int)r, (int)N, (int)ld,
                   cnt, nullptr, nullptr, st);
    hipLaunchKernelGGL(k_ek_delta, dim3(cnt), dim3(NT), 0, st, ek->Xs.as<double>(), ld * ld, (int)N,
                       (int)ld, ek->Lz.as<double>(), ek->q, d_dev + (size_t)p0 * r, (int)r,
                       ek->cstd.as<double>(), delta_dev + p0, nrm_dev ? nrm_dev + 2 * p0 : nullptr);
    LYAP_HIP(hipGetLastError());
  }
}

void ek_solve_impl(lyap_ek_s* ek, int64_t P, const double* d_dev, const lyap_solve_opts* opts,
                   double* W_dev, double* delta_dev, double* nrm_dev, lyap_result* res) {
  LYAP_REQUIRE(ek->proj, LYAP_E_INVAL, "ek_set_level was not called");
  LYAP_REQUIRE(P >= 1 && d_dev && W_dev && delta_dev && res, LYAP_E_INVAL, "bad argument");
  const lyap_status s = smw_solve_batch(ek->proj, P, d_dev, opts, W_dev, res, nullptr, 0, ek->st);
  if (s != LYAP_OK) throw Error{s, std::string("projected solve: ") + lyap_last_error()};
  ek_delta_impl(ek, P, d_dev, W_dev, delta_dev, nrm_dev);
  LYAP_HIP(hipStreamSynchronize(ek->st));
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
  LYAP_TRY(ek_set_level_impl(ek, m, proj_opts));
  return LYAP_OK;
}

lyap_status ek_solve(lyap_ek ek, int64_t P, const double* d_dev, const lyap_solve_opts* opts,
                     double* W_dev, double* delta_dev, double* norms_dev, lyap_result* res_host) {
  if (!ek) return LYAP_E_INVAL;
  LYAP_TRY(ek_solve_impl(ek, P, d_dev, opts, W_dev, delta_dev, norms_dev, res_host));
  return LYAP_OK;
}

lyap_status ek_sweep(lyap_ek ek, int64_t P, const double* d_host, const lyap_solve_opts* opts,
                     const lyap_seed_opts* proj_opts, double eps, int32_t m_max,
                     int32_t check_every, lyap_ek_result* out) {
  if (!ek || P < 1 || !d_host || !out || !(eps > 0) || m_max < 1 || check_every < 1)
    return LYAP_E_INVAL;
  LYAP_TRY({
    const long r = ek->r;
    for (int64_t i = 0; i < P * r; ++i)
      LYAP_REQUIRE(std::isfinite(d_host[i]), LYAP_E_INVAL, "non-finite parameter");
    for (int64_t i = 0; i < P; ++i) {
      out[i].status = LYAP_E_NOCONV;
      out[i].level = 0;
      out[i].dim = 0;
      out[i].iters = 0;
      out[i].delta = NAN;
      out[i].trace = NAN;
    }
    std::vector<int64_t> todo(P);
    for (int64_t i = 0; i < P; ++i) todo[i] = i;
    std::vector<double> dl, delta;
    std::vector<lyap_result> res;
    int m = 1;
    while (!todo.empty() && m <= m_max) {
      ek_set_level_impl(ek, m, proj_opts);
      const int64_t R = (int64_t)todo.size();
      dl.resize((size_t)R * r);
      for (int64_t t = 0; t < R; ++t)
        std::memcpy(&dl[(size_t)t * r], d_host + (size_t)todo[t] * r, sizeof(double) * r);
      if (ek->ddev.bytes < dl.size() * sizeof(double)) ek->ddev.alloc(dl.size() * sizeof(double));
      const size_t wb = (size_t)R * r * ek->dim * sizeof(double);
      if (ek->Wbuf.bytes < wb) ek->Wbuf.alloc(wb);
      if (ek->dl.bytes < (size_t)R * sizeof(double)) ek->dl.alloc((size_t)R * sizeof(double));
      LYAP_HIP(hipMemcpyAsync(ek->ddev.p, dl.data(), dl.size() * sizeof(double),
                              hipMemcpyHostToDevice, ek->st));
      res.resize(R);
      ek_solve_impl(ek, R, ek->ddev.as<double>(), opts, ek->Wbuf.as<double>(), ek->dl.as<double>(),
                    nullptr, res.data());
      delta.resize(R);
      LYAP_HIP(hipMemcpyAsync(delta.data(), ek->dl.p, (size_t)R * sizeof(double),
                              hipMemcpyDeviceToHost, ek->st));
      LYAP_HIP(hipStreamSynchronize(ek->st));
      std::vector<int64_t> rest;
      const bool last = ek->q == 0;  // the space is invariant: the projection is exact
      for (int64_t t = 0; t < R; ++t) {
        lyap_ek_result& o = out[todo[t]];
        o.iters += res[t].iters;
        o.level = ek->level;
        o.dim = ek->dim;
        o.delta = delta[t];
        o.trace = res[t].trace;
        if (res[t].status != LYAP_OK) {
          // the projected solve failed at this level: kept for the next one,
          // its status stands if no later level accepts it
          o.status = res[t].status;
          rest.push_back(todo[t]);
          continue;
        }
        if (delta[t] <= eps || last) {
          o.status = LYAP_OK;
        } else {
          o.status = LYAP_E_NOCONV;
          rest.push_back(todo[t]);
        }
      }
      todo.swap(rest);
      if (last) break;
      m = ek->level + check_every;
    }
  });
  return LYAP_OK;
}

lyap_status ek_info(lyap_ek ek, lyap_ek_info* o) {
  if (!ek || !o) return LYAP_E_INVAL;
  o->n = ek->n;
  o->r = ek->r;
  o->level = ek->level;
  o->dim = ek->dim;
  o->blocks = ek->nblocks();
  o->basis_cols = (int64_t)(ek->Q.size() / ek->n);
  o->exhausted = ek->exhausted ? 1 : 0;
  o->proj_basis = ek->proj ? ek->proj->basis : -1;
  o->proj_cond = ek->proj ? ek->proj->cond_est : 0.0;
  o->basis_seconds = ek->basis_seconds;
  o->level_seconds = ek->level_seconds;
  return LYAP_OK;
}

lyap_status ek_release(lyap_ek ek) {
  if (!ek) return LYAP_E_INVAL;
  delete ek;
  return LYAP_OK;
}

}  // extern "C"
