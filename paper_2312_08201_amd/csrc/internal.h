// Internal structures of the lyapsmw library.
//
// Real form of the complex eigenbasis.  A0 = Q0 Lambda0 Q0^-1 (Section 2.1)
// with complex-conjugate eigenpairs.  Every quantity the method needs in
// eigen-coordinates (Q0^-1 U, V^T Q0, Y Q0^-T, the Cauchy contraction ...) is
// a complex vector whose entries for lambda and conj(lambda) are conjugate.
// It is stored as a real "rho-vector" of length n: for the k-th pair
// (Im lambda_k > 0) the entries 2k, 2k+1 hold the real and imaginary part of
// the lambda_k entry; real eigenvalues follow at 2h, 2h+1, ...  Products of
// two such vectors are complex on pair slots and real elsewhere.
//
// S (n x n, real) holds the eigenvectors in the same order:
// S[:, 2k] = Re q_k, S[:, 2k+1] = Im q_k, S[:, 2h+m] = real eigenvector m.
// Then Q0^-1 row k = (S^-1 row 2k - i S^-1 row 2k+1) / 2, which gives
//   rho(Y Q0^-T) = (Y S^-T) * sig,   sig = (1/2, -1/2, ..., 1, ...)
//   Y           = (rho(Yhat) * sigp) S^T,  sigp = (2, -2, ..., 1, ...)
//   rho(V^T Q0) = V^T S.
#pragma once

#include <mutex>

#include "common.h"

struct lyap_seed_s {
  int64_t n = 0, r = 0, s = 0, h = 0, ld = 0;
  int basis = LYAP_BASIS_EIG;
  double cond_est = 0, min_lam_sum = 0, max_re = 0, t0 = 0, factor_seconds = 0;
  double t0_unrefined = 0;  // t0 before the refinement of the right-hand-side quantities
  int seed_refine = 0;      // refinement steps applied to t0, c0, Gamma (eigen basis)
  // relative forward error of the eigenbasis route, |t0_unrefined - t0| / |t0|
  // (with a floor of 4 unit roundoffs), NaN when no refinement measured it
  double eps_seed = NAN;
  hipStream_t stream = nullptr;
  int device = 0;

  // persistent device data (double unless noted; n-vectors have stride ld, zero pad)
  lyap::DevBuf lam;     // 2 x ld: Re / Im of the eigenvalue belonging to each rho slot
  lyap::DevBuf Mc;      // ld x ld: real Cauchy operator, rho(x L) = rho(x) Mc
  lyap::DevBuf Mc32;    // ld x ld float copy
  lyap::DevBuf Mcb;     // 2 planes ld x ld bf16 (hi, lo) of Mc^T
  lyap::DevBuf Tin;     // ld x ld: Tin[m][j] = S^-1[j][m] sig_j   (rho(Y Q0^-T) = Y Tin)
  lyap::DevBuf Tout;    // ld x ld: Tout[j][m] = sigp_j S[m][j]     (Y = rho(Yhat) Tout)
  lyap::DevBuf Uh;      // r x ld  rho(Q0^-1 U)^T
  lyap::DevBuf Vh;      // r x ld  rho(V^T Q0)
  lyap::DevBuf K1;      // r*r x ld: K1[a][b] = rho((Vh_a o Uh_b) L)
  lyap::DevBuf c0;      // r x ld: rho(V^T X0 Q0^-T)
  lyap::DevBuf gam;     // r x ld: trace(E X) = t0 + sum_b <gam_b, rho(Yhat_b)>
  lyap::DevBuf Gam;     // r x ld: physical Gamma^T (trace = t0 + 2 <Gamma^T, Y>)
  lyap::DevBuf T, Tt;   // Schur basis only: quasi-triangular T and T^T (ld x ld)
  lyap::DevBuf Bh;      // s x ld: B^T Tin (full solutions only)
  lyap::DevBuf Kd;      // Schur basis, small n: dense capacitance operator (r ld x r ld)
  bool projected = false;  // right-hand side given through V^T X0 (no B)
  // rank-pbar TSVD of the dense coupling (preconditioner of eq:prec), r*ld x 128
  int pbar = 0;
  double tsvd_sigma_ratio = 0;  // sigma_(pbar+1) / sigma_1 of the coupling
  lyap::DevBuf TsM, TsN;  // Mt, Nt (row-major r*ld x 128, columns >= pbar zero)
  lyap::DevBuf TsNt;      // Nt^T (128 x r*ld)
  lyap::DevBuf scratch; // grown on demand by lyap_seed_apply / trace_EX
  size_t scratch_bytes = 0;
  // smw_solve_batch keeps its engine (buffers and captured step graphs) for the
  // next call with the same slots, queue length, options and solution store;
  // sol_buf is the solution store when the caller passes no workspace.
  std::mutex cache_mu;
  void* eng_cache = nullptr;
  void (*eng_cache_free)(void*) = nullptr;
  size_t (*eng_cache_bytes)(const void*) = nullptr;
  lyap::DevBuf sol_buf;

  ~lyap_seed_s() {
    if (eng_cache && eng_cache_free) eng_cache_free(eng_cache);
  }

  size_t device_bytes() const {
    return lam.bytes + Mc.bytes + Mc32.bytes + Mcb.bytes + Tin.bytes + Tout.bytes + Uh.bytes +
           Vh.bytes + K1.bytes + c0.bytes + gam.bytes + Gam.bytes + T.bytes + Tt.bytes + Bh.bytes + Kd.bytes +
           TsM.bytes + TsN.bytes + TsNt.bytes + scratch.bytes + sol_buf.bytes +
           (eng_cache && eng_cache_bytes ? eng_cache_bytes(eng_cache) : 0);
  }
};

namespace lyap {

// ---- elementwise helpers on rho-vectors (launchers, seed.hip) ----
// out[(i*nb + j)] = a_i o b_j  (rho-complex product), rows of length ld
void hadamard_outer(double* out, const double* a, long lda, int na, const double* b, long ldb,
                    int nb, int h, int n, int ld, hipStream_t s);
// out[g] (+)= scale * sum_{t < G} w_t o H[g*G + t]   for g < ngroups
void contract_groups(double* out, const double* H, long ldh, const double* w, long ldw, int ngroups,
                     int G, int h, int n, int ld, double scale, bool accumulate, hipStream_t s);
// deterministic dot products: out[p] = base + scale * sum_k x[p*stride + k] * y[(p % ymod)*... ]
void batched_dot(double* out, const double* X, long ldx, const double* Y, long ldy, int rows_per,
                 int count, int n, double base, double scale, hipStream_t s);
void convert_f64_f32(float* out, const double* in, long count, hipStream_t s);

// ---- projected seeds (seed.hip) ----
// A seed whose right-hand side is known only through V^T X0 (c0t, host r x n
// row-major) and t0 = trace(E X0): the Galerkin-projected equations of the
// extended Krylov framework, where X0 is the full seed solution seen through
// the basis.  No stability requirement on A0 (only lambda_i + lambda_j != 0).
struct ProjRhs {
  const double* c0t;
  double t0;
};
lyap_seed_s* factor_projected(int64_t n, int64_t r, const double* A0, const double* U,
                              const double* V, const double* E, const ProjRhs& proj,
                              const lyap_seed_opts* opts, hipStream_t stream);

// ---- the seed apply (apply.hip): G = V^T X, A0 X + X A0^T = U Y + Y^T U^T, FP64 ----
void seed_apply64(lyap_seed_s* sd, long long batch, const double* Y, double* G, hipStream_t st);

// ---- engines owned inside the library (engine.hip) ----
// An engine with queue and solution store for up to P_cap parameters; batches
// of any size up to that run on it after a reset (see smw_solve_batch).
lyap_engine_s* engine_batch_create(lyap_seed_s* sd, long long P_cap, const lyap_solve_opts* opts,
                                   hipStream_t st, double* sol);
void engine_batch_reset(lyap_engine_s* E, hipStream_t st);
void engine_batch_destroy(lyap_engine_s* E);
bool engine_batch_fits(const lyap_engine_s* E, long long P, const lyap_solve_opts* opts);
void engine_batch_run(lyap_engine_s* E, long long P, const double* d_dev, double* Y_dev,
                      lyap_result* res_host);

// ---- Schur basis (schur.hip) ----
// T Xs + Xs T^T = C per problem; C dense (Cd, row-major) or F G^T + G F^T
// (F: k rows, shared or fstride apart per problem; G: k rows per problem).
// X stored column by column.
void trilyap_launch(const double* T, const double* Tt, double* X, long xstride, const double* Cd,
                    long cstride, const double* F, const double* G, long gstride, int k, int n,
                    int ld, int count, const int* list, const int* count_dev, hipStream_t st,
                    long fstride = 0);
// Tile-blocked solver (schur.hip) for count problems sharing T: X_b
// (row-major, xrows >= n rows of ld, problems xrows ld apart, rows >= n
// zero) with T X_b + X_b T^T = Cd + F_b G_b^T + G_b F_b^T (Cd dense symmetric,
// shared, or null; F_b, G_b k rows of ld, fstride / gstride apart, 0 =
// shared).  Allocates its workspace; synchronises the stream.
void trilyap_blocked(const double* T, const double* Tt, int n, int ld, const double* Cd,
                     const double* F, long fstride, const double* G, long gstride, int k,
                     long count, long xrows, double* X, hipStream_t st);
// out_p[a] = sum_m Vt[a][m] X_p[m][:]
void project_launch(const double* Vt, const double* X, long xstride, double* out, long ostride,
                    int r, int n, int ld, int count, const int* list, const int* count_dev,
                    hipStream_t st);
// Dense capacitance operator of a Schur-basis seed (sd->Kd), see schur.hip.
void schur_dense_operator(lyap_seed_s* sd, hipStream_t st);
void gemm64_rm(const double* A, long lda, const double* B, long ldb, double* C, long ldc, long M,
               long N, long K, long Nstore, hipStream_t s);

// ---- dense solves in the real eigenbasis (full.hip) ----
// In place on C (ld x ld, real eigen coordinates, no sig scaling): the
// block-diagonal equation Lambda X + X Lambda^T = C, or with adjoint
// Lambda^T X + X Lambda = C (Lambda from the seed's lam).
void blockdiag_dense_launch(double* C, const double* lam, int n, int h, int ld, bool adjoint,
                            hipStream_t st);
// out = alpha (M + M^T) + beta C on the leading n x n block, zero outside it
void sym_combine_launch(double* out, const double* M, const double* C, double alpha, double beta,
                        int n, int ld, hipStream_t st);
// out = a + b over count doubles
void add_launch(double* out, const double* a, const double* b, long count, hipStream_t st);

}  // namespace lyap
