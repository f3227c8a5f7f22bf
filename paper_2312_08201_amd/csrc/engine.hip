// Online stage (Section 2.1, Table 1 right column): the batched Krylov engine.
//
// Every busy slot holds one parameter sample p and advances one Krylov step
// per engine step.  A step is a fixed sequence of launches (captured once as
// a HIP graph):
//   k_prep      z = P^-1 v_j (Arnoldi step) or z = P^-1 u (residual step);
//               the iterate u is kept before preconditioning, y = P^-1 u
//   k_formX     rows (p, a, b) of the Cauchy GEMM: Vh_a o z_b
//   GEMM        H = X * Mc  (MFMA, FP64 or FP32 / split-BF16)
//   k_epilogue  w = z - D (sum_b z_b o K1_ab + sum_b Uh_b o H_pab)
//   k_krylov    one workgroup per slot: CGS2 orthogonalisation with
//               wavefront reductions, Givens update in FP64, restart with a
//               true FP64 residual, convergence, result write-out and
//               admission of the next queued parameter (device-side queue).
//   k_claim_lists  queue claims of the free slots and the compacted lists of
//               the slots that need an FP64 or a low-precision product in the
//               next step (device counts), then k_admit
//
// The capacitance system is the n*r reduced form of eq:SMW_linearsystem,
// scaled by D so that d = 0 is allowed:  (I - D K) y = D c0,
// K(y) = Vh (L o (Uh y + y^T Uh^T)) in eigen-coordinates.  The right
// preconditioner is the exact block-diagonal part of eq:prec: per eigen slot
// j the r x r block I - D K1[:, :, j] (complex on conjugate pairs).
// Mixed precision: Arnoldi products use the low-precision GEMM, every
// restart evaluates the residual with the FP64 GEMM (iterative refinement).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <tuple>
#include <mutex>
#include <type_traits>

#include "internal.h"

namespace lyap {

constexpr int kPrecRank = 8;     // block preconditioner up to r = 8
constexpr int kMaxRecycle = 16;  // recycle space dimension bound
constexpr int kMaxBasis = kMaxRestart + kMaxRecycle;

enum Phase : int { PH_FREE = 0, PH_ARNOLDI = 1, PH_RESTART = 2, PH_RECYC = 3, PH_NEWSPACE = 4 };

// per-slot integer state (KCUR: valid recycle vectors, RJ: next one to
// rebuild for a new parameter, BANK: which of the two U/C banks is current)
enum SI : int {
  SI_PHASE = 0, SI_J, SI_ITERS, SI_CYCLES, SI_REFINE, SI_QPOS, SI_KCUR, SI_RJ, SI_BANK, SI_CAPSET,
  SI_PINV, SI_COMB, SI_PASSB, SI_CLAIM, SI_N
};
constexpr int kPbarMax = 64;  // TSVD rank bound of the preconditioner
constexpr int kTsvdGrid = 256;  // workgroup budget of the skinny TSVD GEMM (split-K)
// Split-K partials (the TSVD GEMM, one column tile): a launch of G
// workgroups writes at most G row tiles of partials; its buffer holds
// kTsvdGrid row tiles.
// The Cauchy GEMMs run stream-K (sk_plan) on kSkGridUnit x {2, 4}
// workgroups (two or four per CU of a 256-CU device; the autotuner picks).
// Their partial buffers hold the segments of the largest candidate grid at
// any active row count, for every K-tile depth a launch may use.
constexpr int kSkGridUnit = 256;
constexpr int kSkGridMults[2] = {2, 4};
inline long long cauchy_part_rows(long long rows_pad, long long ld, GemmType type) {
  const int nks[2] = {type == GemmType::F64 ? 8 : 16, type == GemmType::F64 ? 16 : 32};
  long long rows = 0;
  for (int mult : kSkGridMults)
    for (int bk : nks) {
      if (type == GemmType::BF16X3 && bk != 32) continue;
      rows = std::max(rows, sk_part_rows(rows_pad, (int)(ld / kGemmBN), mult * kSkGridUnit,
                                         (int)(ld / bk)));
    }
  return rows;
}
// per-slot double state
enum SD : int { SD_BNORM = 0, SD_BETA, SD_N };

struct DevResult {  // one per queue position
  int status, iters, cycles, refines;
  double relres, trace, err_est;
  long long tag;
  int valid, pad;
};

struct EngineArgs {
  // seed
  const double* Uh;
  const double* Vh;
  const double* K1;
  const double* c0;
  const double* gam;
  double t0;
  double eps_seed;  // relative forward error of the seed's eigenbasis route (NaN: unknown)
  int n, h, ld, r;
  int NV;  // per-slot vector stride: r * ld padded to a multiple of 512
  // engine
  int S, m, max_iter, max_refine, use_precond, mixed;
  double tol, inner_tol;
  int* si;          // S x SI_N
  double* sdv;      // S x SD_N
  double* d;        // S x r
  double* R;        // S x m x (m+1)  rotated Hessenberg columns
  double* g;        // S x (m+1)
  double* cs;       // S x m
  double* sn;       // S x m
  double* V;        // S x (m+1) x N
  double* x;        // S x N
  double* z;        // S x N
  double* w;        // S x N
  double* Pinv;     // S x r*r x ld
  int* lists;       // [0..S): FP64 list, [S..2S): low-precision list, [2S], [2S+1] counts
  // queue (ring of capacity Q) and results
  const double* qd;        // Q x r
  const long long* qtag;   // Q
  int* qctl;               // [0] head, [1] tail, [2] done count
  DevResult* res;          // Q
  int Q;
  double* sol;             // optional: solutions by tag, stride N (rho form)
  long long sol_cap;
  // recycling (GCRO-DR); kmax = 0 disables it
  int kmax;
  double* Ur;   // S x 2 banks x kmax x NV: U with A P^-1 U = C
  double* Cr;   // S x 2 banks x kmax x NV: C, orthonormal columns
  double* Bk;   // S x kmax x m: C^T A P^-1 v_j of the current cycle
  double* Hr;   // S x m x (m+1): unrotated Hessenberg columns
  double* Fs;   // S x kRecScratch: recycle-update work matrix
  // low-rank coupling of the preconditioner (TSVD rank pbar; 0 disables it)
  int pbar, Ks;         // Ks = r * ld
  const double* TsM;    // Ks x 128: Mt
  const double* TsN;    // Ks x 128: Nt
  double* Cpinv;        // S x 64 x 64: (I - Mt^T B^-1 D Nt)^-1 per slot
  double* Yc;           // list-compacted y = B^-1 v rows (Ks)
  double* Tbuf;         // list rows x 128: Mt^T y
  double* Tpart;        // split-K partials of Tbuf
  double* Sc;           // list rows x 128: Cp^-1 Mt^T y
  double* Qc;           // list rows x Ks: Nt Cp^-1 Mt^T y
  // split orthogonalisation (restarted GMRES): per slot and chunk of the
  // slot vector, the chunk's partial projections and norms
  int nchunk;           // NV / (2 x orth workgroup size)
  double* orth1;        // S x nchunk x kPart: <v_k, w> chunk sums (k <= j), ||w||^2 last
  double* orth1b;       // the same after the first pass
  double* orth2;        // S x nchunk: ||w||^2 chunk sums after the second pass
  double* ycoefs;       // S x (kMaxRestart + 1): cycle-end coefficients y (u += V y)
  // delayed reorthogonalisation (dcgs = 1, see k_orth_a): chunk partials of
  // the one projection pass, the update coefficients of the second pass and
  // the unrotated Hessenberg columns
  int dcgs;
  int vf32;             // 1: the basis is stored in FP32 (Vf), see basis_f32
  float* Vf;            // S x (m+1) x NV when vf32
  double* orthA;        // S x nchunk x kPartA
  double* coefB;        // S x kPartA: a (m), b (m), 1 / beta, z
  double* Hu;           // S x m x (m + 1)
};

__device__ inline double* rec_u(const EngineArgs& A, int s, int bank, int l) {
  return A.Ur + (((long)s * 2 + bank) * A.kmax + l) * (long)A.NV;
}
__device__ inline double* rec_c(const EngineArgs& A, int s, int bank, int l) {
  return A.Cr + (((long)s * 2 + bank) * A.kmax + l) * (long)A.NV;
}

// ---------------------------------------------------------------------------
// reductions (64-wide wavefronts, 256-thread workgroups)
// ---------------------------------------------------------------------------
constexpr int KT = 256;   // threads of the per-slot and grid-stride kernels
constexpr int KK = 1024;  // threads of the Krylov kernel (16 wavefronts per slot)

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// sum over the workgroup of NV values per thread, result visible to all
// threads (lds: NV * waves doubles; waves summed in fixed order)
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) lds[wave * NV + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += lds[w * NV + i];
    v[i] = t;
  }
  __syncthreads();
}

__device__ inline double block_sum1(double v, double* lds) {
  double a[1] = {v};
  block_sum<1>(a, lds);
  return a[0];
}

// a slot's phase and Arnoldi index in one load (adjacent, 8-byte aligned), so
// that the index does not wait for the phase test
static_assert(SI_J == SI_PHASE + 1 && SI_PHASE % 2 == 0 && (SI_N * 4) % 8 == 0,
              "phase and index load as one int2");
__device__ inline int2 phase_j(const int* si_slot) {
  return *reinterpret_cast<const int2*>(si_slot + SI_PHASE);
}

// unit u: conjugate pair u < h (slots 2u, 2u+1) or real eigenvalue (slot u + h)
__device__ inline int uslot(int u, int h, bool& pr) {
  pr = u < h;
  return pr ? 2 * u : u + h;
}

// at(0) + at(1) + ... + at(n - 1), added in index order, with eight loads in
// flight at a time (per-chunk partials of one slot: n is small, and a plain
// loop would wait for every load before issuing the next)
template <class F>
__device__ inline double chunk_sum(int n, F&& at) {
  double acc = 0.0;
  for (int q0 = 0; q0 < n; q0 += 8) {
    double v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = q0 + e < n ? at(q0 + e) : 0.0;
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (q0 + e < n) acc += v[e];
  }
  return acc;
}

// out(e, in(e)) for e = threadIdx.x, threadIdx.x + blockDim.x, ... < n, with
// the loads of eight consecutive steps issued before their stores (a plain
// loop waits for each load, since the compiler cannot move a load above a
// store that may alias it)
template <class In, class Out>
__device__ inline void strided_map(int n, In&& in, Out&& out) {
  const int bd = (int)blockDim.x;
  for (int e0 = threadIdx.x; e0 < n; e0 += 8 * bd) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = e0 + q * bd < n ? in(e0 + q * bd) : 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (e0 + q * bd < n) out(e0 + q * bd, v[q]);
  }
}

// f(std::integral_constant<int, R>) with R = r for r <= 4 and R = 0 (r read at
// run time) otherwise: per-unit loops over r unroll, so their loads issue
// together instead of one round trip per loop step.
template <class F>
__device__ inline void dispatch_r(int r, F&& f) {
  switch (r) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    default: f(std::integral_constant<int, 0>{}); break;
  }
}

// z_a[u] = sum_b P[a][b][u] o v_b[u] for one slot (all a), units u0 + threadIdx.x,
// u0 + threadIdx.x + ustride, ... (default: all units by this workgroup);
// RT: r at compile time (0: read from A)
template <int RT = 0, class ST = double>
__device__ inline void apply_pinv(const EngineArgs& A, int s, const ST* v, double* zout,
                                  bool accumulate, const double* vscale = nullptr, int u0 = 0,
                                  int ustride = 0) {
  const int r = RT > 0 ? RT : A.r, ld = A.ld, nu = A.n - A.h;
  const double* P = A.Pinv + (long)s * r * r * ld;
  if (ustride == 0) ustride = blockDim.x;
  for (int u = u0 + threadIdx.x; u < nu; u += ustride) {
    bool pr;
    const int q = uslot(u, A.h, pr);
#pragma unroll
    for (int a = 0; a < r; ++a) {
      double sr = 0, si = 0;
#pragma unroll
      for (int b = 0; b < r; ++b) {
        const double* pb = P + (long)(a * r + b) * ld;
        const ST* vb = v + (long)b * ld;
        if (pr) {
          const double f = vscale ? vscale[b] : 1.0;
          const double pr_ = pb[q], pi_ = pb[q + 1], vr = f * (double)vb[q],
                       vi = f * (double)vb[q + 1];
          sr += pr_ * vr - pi_ * vi;
          si += pr_ * vi + pi_ * vr;
        } else {
          sr += pb[q] * (vscale ? vscale[b] : 1.0) * (double)vb[q];
        }
      }
      double* za = zout + (long)a * ld;
      if (accumulate) {
        za[q] += sr;
        if (pr) za[q + 1] += si;
      } else {
        za[q] = sr;
        if (pr) za[q + 1] = si;
      }
    }
  }
}

// (I - D K1_q)^-1 for one eigen slot q (complex r x r on a conjugate pair),
// Gauss-Jordan with partial pivoting; R is the compile-time bound of r.
template <int R>
__device__ inline void block_inverse(const EngineArgs& A, const double* dsh, int q, bool pr,
                                     double* P, int r = R) {
  double Mr[R * R], Mi[R * R], Ir[R * R], Ii[R * R];
  const int ld = A.ld;
#pragma unroll
  for (int a = 0; a < R; ++a)
#pragma unroll
    for (int b = 0; b < R; ++b) {
      if (a >= r || b >= r) continue;
      const double* k = A.K1 + (long)(a * r + b) * ld;
      Mr[a * R + b] = (a == b ? 1.0 : 0.0) - dsh[a] * k[q];
      Mi[a * R + b] = pr ? -dsh[a] * k[q + 1] : 0.0;
      Ir[a * R + b] = a == b ? 1.0 : 0.0;
      Ii[a * R + b] = 0.0;
    }
#pragma unroll
  for (int c = 0; c < R; ++c) {
    if (c >= r) break;
    int piv = c;
    double best = -1;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if (i < c || i >= r) continue;
      const double mag = fabs(Mr[i * R + c]) + fabs(Mi[i * R + c]);
      if (mag > best) {
        best = mag;
        piv = i;
      }
    }
    if (piv != c) {
#pragma unroll
      for (int b = 0; b < R; ++b) {
        double t;
        t = Mr[c * R + b]; Mr[c * R + b] = Mr[piv * R + b]; Mr[piv * R + b] = t;
        t = Mi[c * R + b]; Mi[c * R + b] = Mi[piv * R + b]; Mi[piv * R + b] = t;
        t = Ir[c * R + b]; Ir[c * R + b] = Ir[piv * R + b]; Ir[piv * R + b] = t;
        t = Ii[c * R + b]; Ii[c * R + b] = Ii[piv * R + b]; Ii[piv * R + b] = t;
      }
    }
    const double pr_ = Mr[c * R + c], pi_ = Mi[c * R + c];
    const double den = pr_ * pr_ + pi_ * pi_;
    const double ivr = pr_ / den, ivi = -pi_ / den;
#pragma unroll
    for (int b = 0; b < R; ++b) {
      double ar = Mr[c * R + b], ai = Mi[c * R + b];
      Mr[c * R + b] = ar * ivr - ai * ivi;
      Mi[c * R + b] = ar * ivi + ai * ivr;
      ar = Ir[c * R + b];
      ai = Ii[c * R + b];
      Ir[c * R + b] = ar * ivr - ai * ivi;
      Ii[c * R + b] = ar * ivi + ai * ivr;
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if (i == c || i >= r) continue;
      const double fr = Mr[i * R + c], fi = Mi[i * R + c];
#pragma unroll
      for (int b = 0; b < R; ++b) {
        Mr[i * R + b] -= fr * Mr[c * R + b] - fi * Mi[c * R + b];
        Mi[i * R + b] -= fr * Mi[c * R + b] + fi * Mr[c * R + b];
        Ir[i * R + b] -= fr * Ir[c * R + b] - fi * Ii[c * R + b];
        Ii[i * R + b] -= fr * Ii[c * R + b] + fi * Ir[c * R + b];
      }
    }
  }
#pragma unroll
  for (int a = 0; a < R; ++a)
#pragma unroll
    for (int b = 0; b < R; ++b) {
      if (a >= r || b >= r) continue;
      double* pb = P + (long)(a * r + b) * ld;
      pb[q] = Ir[a * R + b];
      if (pr) pb[q + 1] = Ii[a * R + b];
    }
}

// (I - D K1_q)^-1 for 4 < r <= 8 by one wavefront: lane 8 i + j holds
// entry (i, j) of the matrix and of its inverse (complex on a conjugate
// pair); Gauss-Jordan with partial pivoting through lane shuffles.
__device__ inline void wave_inverse(const EngineArgs& A, const double* d, int q, bool pr,
                                    double* P, int lane) {
  const int r = A.r, ld = A.ld;
  const int i = lane >> 3, j = lane & 7;
  const bool in = i < r && j < r;
  double mr = 0, mi = 0, ir = 0, ii = 0;
  if (in) {
    const double* k = A.K1 + (long)(i * r + j) * ld;
    mr = (i == j ? 1.0 : 0.0) - d[i] * k[q];
    mi = pr ? -d[i] * k[q + 1] : 0.0;
    ir = i == j ? 1.0 : 0.0;
  }
  for (int c = 0; c < r; ++c) {
    // pivot row: largest |entry| in column c at or below row c
    double mag = (in && j == c && i >= c) ? fabs(mr) + fabs(mi) : -1.0;
    int row = i;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double om = __shfl_xor(mag, o, 64);
      const int orow = __shfl_xor(row, o, 64);
      if (om > mag || (om == mag && orow < row)) {
        mag = om;
        row = orow;
      }
    }
    const int pv = row;
    // swap rows c and pv
    const int src = i == c ? pv * 8 + j : (i == pv ? c * 8 + j : lane);
    mr = __shfl(mr, src, 64);
    mi = __shfl(mi, src, 64);
    ir = __shfl(ir, src, 64);
    ii = __shfl(ii, src, 64);
    // scale row c by 1 / pivot
    const double pr_ = __shfl(mr, c * 8 + c, 64), pi_ = __shfl(mi, c * 8 + c, 64);
    const double den = pr_ * pr_ + pi_ * pi_;
    const double vr = pr_ / den, vi = -pi_ / den;
    if (i == c) {
      double t = mr * vr - mi * vi;
      mi = mr * vi + mi * vr;
      mr = t;
      t = ir * vr - ii * vi;
      ii = ir * vi + ii * vr;
      ir = t;
    }
    // eliminate column c from the other rows
    const double fr = __shfl(mr, i * 8 + c, 64), fi = __shfl(mi, i * 8 + c, 64);
    const double cr = __shfl(mr, c * 8 + j, 64), ci = __shfl(mi, c * 8 + j, 64);
    const double jr = __shfl(ir, c * 8 + j, 64), ji = __shfl(ii, c * 8 + j, 64);
    if (i != c) {
      mr -= fr * cr - fi * ci;
      mi -= fr * ci + fi * cr;
      ir -= fr * jr - fi * ji;
      ii -= fr * ji + fi * jr;
    }
  }
  if (in) {
    double* pb = P + (long)(i * r + j) * ld;
    pb[q] = ir;
    if (pr) pb[q + 1] = ii;
  }
}

// Preconditioner blocks for the slots admitted in this step.  Grid (S,
// chunks): one slot's units are spread over many workgroups, so an admission
// adds one short kernel to the step instead of one long workgroup.
constexpr int kPinvUnitsWave = 32;  // r > 4: units per workgroup (8 per wavefront)
__global__ void __launch_bounds__(KT) k_pinv(EngineArgs A) {
  const int s = blockIdx.x;
  if (A.si[(long)s * SI_N + SI_PINV] == 0) return;
  const int r = A.r, h = A.h, nu = A.n - h;
  const double* d = A.d + (long)s * r;
  double* P = A.Pinv + (long)s * r * r * A.ld;
  if (r <= 4) {
    const int u = blockIdx.y * KT + threadIdx.x;
    if (u >= nu) return;
    bool pr;
    const int q = uslot(u, h, pr);
    switch (r) {
      case 1: block_inverse<1>(A, d, q, pr, P); break;
      case 2: block_inverse<2>(A, d, q, pr, P); break;
      case 3: block_inverse<3>(A, d, q, pr, P); break;
      default: block_inverse<4>(A, d, q, pr, P); break;
    }
  } else {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int uu = wave; uu < kPinvUnitsWave; uu += KT / 64) {
      const int u = blockIdx.y * kPinvUnitsWave + uu;
      if (u >= nu) break;
      bool pr;
      const int q = uslot(u, h, pr);
      wave_inverse(A, d, q, pr, P, lane);
    }
  }
}

static int pinv_chunks(int r, int nu) {
  return r <= 4 ? (nu + KT - 1) / KT : (nu + kPinvUnitsWave - 1) / kPinvUnitsWave;
}

// With r <= 4 and no TSVD part, the blocks of a newly admitted slot are built
// by the next step's k_prep, each thread for the units it then applies them
// to, instead of by k_pinv right after the admission (one launch fewer per
// step).  The TSVD capacitance set up at the admission needs the blocks at
// once, and r > 4 inverts per wavefront: both keep k_pinv.
__host__ __device__ inline bool lazy_pinv(const EngineArgs& A) {
  return A.use_precond && A.r <= 4 && A.pbar == 0;
}
__device__ inline void build_pinv(const EngineArgs& A, int s, int u0, int ustride) {
  const int r = A.r, nu = A.n - A.h;
  const double* d = A.d + (long)s * r;
  double* P = A.Pinv + (long)s * r * r * A.ld;
  for (int u = u0 + threadIdx.x; u < nu; u += ustride) {
    bool pr;
    const int q = uslot(u, A.h, pr);
    switch (r) {
      case 1: block_inverse<1>(A, d, q, pr, P); break;
      case 2: block_inverse<2>(A, d, q, pr, P); break;
      case 3: block_inverse<3>(A, d, q, pr, P); break;
      default: block_inverse<4>(A, d, q, pr, P); break;
    }
  }
}

// Admission of queue entry qp into slot s (whole workgroup): d(p), right-hand
// side b = D c0, v0 = b / ||b||.  The preconditioner blocks (I - D K1_j)^-1
// follow: in the next step's k_prep (see lazy_pinv) or in k_pinv.
__device__ void admit(const EngineArgs& A, int s, int qp, double* lds) {
  const int r = A.r, ld = A.ld, N = r * ld, NV = A.NV, nu = A.n - A.h;
  int* si = A.si + (long)s * SI_N;
  double* sdv = A.sdv + (long)s * SD_N;
  const int qi = qp % A.Q;
  double* d = A.d + (long)s * r;
  __shared__ double dsh[kMaxRank];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  if (threadIdx.x < r) {
    const double v = A.qd[(long)qi * r + threadIdx.x];
    dsh[threadIdx.x] = v;
    d[threadIdx.x] = v;
    if (!isfinite(v)) atomicOr(&bad, 1);
  }
  __syncthreads();
  double* xs = A.x + (long)s * NV;
  double* V0 = A.V + (long)s * (A.m + 1) * NV;
  for (int e = threadIdx.x; e < NV; e += blockDim.x) xs[e] = 0.0;
  if (bad) {
    if (threadIdx.x == 0) {
      DevResult& o = A.res[qi];
      o.status = LYAP_E_NONFINITE;
      o.iters = o.cycles = o.refines = 0;
      o.relres = NAN;
      o.trace = NAN;
      o.err_est = NAN;
      o.tag = A.qtag[qi];
      __threadfence();
      o.valid = 1;
      si[SI_PHASE] = PH_FREE;
      atomicAdd(&A.qctl[2], 1);
    }
    __syncthreads();
    return;
  }
  // b = D c0 ; ||b||
  double acc = 0;
#pragma unroll 8
  for (int e = threadIdx.x; e < N; e += blockDim.x) {
    const double v = dsh[e / ld] * A.c0[e];
    acc += v * v;
  }
  const double bn = sqrt(block_sum1(acc, lds));
  if (bn == 0.0) {
    // D = 0: y = 0 is exact, X(p) = X0; the solution store gets the zero y
    const long long tag0 = A.qtag[qi];
    if (A.sol && tag0 >= 0 && tag0 < A.sol_cap) {
      double* dst = A.sol + tag0 * (long long)N;
      for (int e = threadIdx.x; e < N; e += blockDim.x) dst[e] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      DevResult& o = A.res[qi];
      o.status = LYAP_OK;
      o.iters = o.cycles = o.refines = 0;
      o.relres = 0.0;
      o.trace = A.t0;
      o.err_est = A.eps_seed;
      o.tag = A.qtag[qi];
      __threadfence();
      o.valid = 1;
      si[SI_PHASE] = PH_FREE;
      atomicAdd(&A.qctl[2], 1);
    }
    __syncthreads();
    return;
  }
  // v_0 = b / ||b|| (the FP32 basis of the low-precision modes, else FP64)
  const double inv = 1.0 / bn;
  if (A.vf32) {
    float* V0f = A.Vf + (long)s * (A.m + 1) * NV;
    strided_map(N, [&](int e) { return A.c0[e]; },
                [&](int e, double c) { V0f[e] = (float)(dsh[e / ld] * c * inv); });
  } else {
    strided_map(N, [&](int e) { return A.c0[e]; },
                [&](int e, double c) { V0[e] = dsh[e / ld] * c * inv; });
  }
  if (threadIdx.x == 0) {
    // a slot that kept a recycle space from its previous parameter first
    // rebuilds C = A(p) P(p)^-1 U for the new parameter
    const bool rec = A.kmax > 0 && si[SI_KCUR] > 0;
    si[SI_PHASE] = rec ? PH_RECYC : PH_ARNOLDI;
    si[SI_RJ] = 0;
    si[SI_CAPSET] = A.pbar > 0 ? 1 : 0;
    si[SI_PINV] = A.use_precond ? 1 : 0;
    si[SI_J] = 0;
    si[SI_ITERS] = 0;
    si[SI_CYCLES] = rec ? 0 : 1;
    si[SI_REFINE] = 0;
    si[SI_QPOS] = qp;
    sdv[SD_BNORM] = bn;
    sdv[SD_BETA] = bn;
    A.g[(long)s * (A.m + 1)] = bn;
  }
  __syncthreads();
}

// The last launch before the admission, in one workgroup, after every slot's
// phase for the step is final:
// * queue claims in slot order: free slot s takes queue position head + (the
//   number of free slots before s) while positions remain, written to
//   si[SI_CLAIM] (-1: none); the head moves past the claimed positions.  The
//   slot a parameter lands in (and so its rows in the Cauchy GEMM) is then a
//   function of the submissions alone.  k_admit admits the claims.
// * the slot lists of the next step (stable compaction in slot order): the
//   slots that need an FP64 product (a restart, or any product in FP64 mode)
//   and those that need a low-precision one.  A claimed slot is listed with
//   the phase its admission gives it (Arnoldi, or the recycle rebuild when it
//   keeps a recycle space).  An admission that fails (a non-finite or zero
//   parameter) leaves its slot free but listed for that one step: the step
//   kernels test the phase and skip it, and its Cauchy GEMM rows are wasted
//   work, nothing else.
// Building the lists here saves a launch per step; the counts therefore
// describe the coming step, and the buffer holds empty lists at creation and
// after a reset.
__device__ inline int claim_phase(const EngineArgs& A, const int* si) {
  const int ph = si[SI_PHASE];
  if (ph != PH_FREE || si[SI_CLAIM] < 0) return ph;
  return A.kmax > 0 && si[SI_KCUR] > 0 ? PH_RECYC : PH_ARNOLDI;
}

__global__ void __launch_bounds__(1024) k_claim_lists(EngineArgs A) {
  __shared__ int cnt[1024], c64[1024], clo[1024];
  const int S = A.S, tid = threadIdx.x;
  const int per = (S + blockDim.x - 1) / blockDim.x;
  const int s0 = tid * per, s1 = min(S, s0 + per);
  int n = 0;
  for (int t = s0; t < s1; ++t) n += A.si[(long)t * SI_N + SI_PHASE] == PH_FREE;
  cnt[tid] = n;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {  // inclusive scan
    const int v = tid >= off ? cnt[tid - off] : 0;
    __syncthreads();
    cnt[tid] += v;
    __syncthreads();
  }
  const int head = A.qctl[0], tail = A.qctl[1];
  int pos = head + cnt[tid] - n;
  int n64 = 0, nlo = 0;
  for (int t = s0; t < s1; ++t) {
    int* si = A.si + (long)t * SI_N;
    if (si[SI_PHASE] == PH_FREE) {
      si[SI_CLAIM] = pos < tail ? pos : -1;
      ++pos;
    }
    si[SI_COMB] = 0;  // this step's cycle ends are combined
    si[SI_PINV] = 0;  // the blocks of this step's admissions are built (k_prep or k_pinv)
    const int ph = claim_phase(A, si);
    const bool arn = ph == PH_ARNOLDI || ph == PH_RECYC;
    if (ph == PH_RESTART || (arn && !A.mixed)) ++n64;
    else if (arn) ++nlo;
  }
  if (tid == blockDim.x - 1) {
    const int total = cnt[tid];
    A.qctl[0] = head + min(total, max(tail - head, 0));
  }
  // inclusive scan of the per-thread list counts
  c64[tid] = n64;
  clo[tid] = nlo;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    const int a = tid >= off ? c64[tid - off] : 0;
    const int b = tid >= off ? clo[tid - off] : 0;
    __syncthreads();
    c64[tid] += a;
    clo[tid] += b;
    __syncthreads();
  }
  if (tid == blockDim.x - 1) {
    A.lists[2 * S] = c64[tid];
    A.lists[2 * S + 1] = clo[tid];
    A.lists[2 * S + 2] = c64[tid] + clo[tid];
  }
  int o64 = c64[tid] - n64, olo = clo[tid] - nlo;
  for (int t = s0; t < s1; ++t) {
    const int ph = claim_phase(A, A.si + (long)t * SI_N);
    const bool arn = ph == PH_ARNOLDI || ph == PH_RECYC;
    if (ph == PH_RESTART || (arn && !A.mixed)) A.lists[o64++] = t;
    else if (arn) A.lists[S + olo++] = t;
  }
}

// Result of slot s.  err_est, the estimated relative error of the trace:
// twice the first-order estimate of the two error sources (the factor covers
// the crudeness of kappa; measured errors on the parity workloads stayed below it):
//   eps_seed (max(1, |t0| / |t|) + kappa (1 + ||D K y|| / ||b||))
//        the seed's eigenbasis route: eps_seed is its relative forward error,
//        measured once per seed by the refinement of t0; it enters t0 (scaled
//        to |t|) and, through the capacitance operator that is not refined,
//        the solve: an operator error of relative size eps_seed perturbs the
//        system by about eps_seed ||D K y|| (= eps_seed ||y - b||), amplified by
//        the condition number of the preconditioned system
//   + kappa relres
//        the capacitance residual left by the Krylov solve
// kappa = the ratio of the largest to the smallest diagonal entry of the last
// cycle's triangular factor (at least 1): an estimate of that condition number.
__device__ void finish(const EngineArgs& A, int s, int status, double relres, double* lds) {
  const int r = A.r, ld = A.ld, N = r * ld;
  int* si = A.si + (long)s * SI_N;
  // the solution y = P^-1 u, formed by this step's prep for the residual
  const double* xs = A.z + (long)s * A.NV;
  const double* ds = A.d + (long)s * r;
  double sums[3] = {0.0, 0.0, 0.0};  // <gam, y>, ||y - b||^2, ||b||^2 with b = D c0
#pragma unroll 8
  for (int e = threadIdx.x; e < N; e += blockDim.x) {
    const double y = xs[e], b = ds[e / ld] * A.c0[e];
    sums[0] += A.gam[e] * y;
    sums[1] += (y - b) * (y - b);
    sums[2] += b * b;
  }
  block_sum<3>(sums, lds);
  const double tr = A.t0 + sums[0];
  // strength of the low-rank correction: (I - D K) y = b gives D K y = y - b
  const double corr = sums[2] > 0.0 ? sqrt(sums[1] / sums[2]) : 0.0;
  const int qp = si[SI_QPOS];
  const int qi = qp % A.Q;
  const long long tag = A.qtag[qi];
  if (A.sol && tag >= 0 && tag < A.sol_cap) {
    double* dst = A.sol + tag * (long long)N;
    strided_map(N, [&](int e) { return xs[e]; }, [&](int e, double v) { dst[e] = v; });
  }
  // largest and smallest |R_kk| of the last cycle over the first wave
  __shared__ double kap_sh;
  if (threadIdx.x < 64) {
    const int jl = min(si[SI_J], A.m);
    const double* Rs = A.R + (long)s * A.m * (A.m + 1);
    double dmax = 0.0, dmin = INFINITY;
    for (int k = threadIdx.x; k < jl; k += 64) {
      const double v = fabs(Rs[(long)k * (A.m + 1) + k]);
      dmax = fmax(dmax, v);
      dmin = fmin(dmin, v);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
      dmin = fmin(dmin, __shfl_xor(dmin, o, 64));
    }
    if (threadIdx.x == 0) kap_sh = (jl > 0 && dmin > 0.0) ? fmax(1.0, dmax / dmin) : 1.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    DevResult& o = A.res[qi];
    o.status = status;
    o.iters = si[SI_ITERS];
    o.cycles = si[SI_CYCLES];
    o.refines = si[SI_REFINE];
    o.relres = relres;
    o.trace = tr;
    {
      const double kappa = kap_sh;
      o.err_est = 2.0 * (A.eps_seed * (fmax(1.0, fabs(A.t0) / fabs(tr)) + kappa * (1.0 + corr)) +
                         kappa * relres);
    }
    o.tag = tag;
    __threadfence();
    o.valid = 1;
    si[SI_PHASE] = PH_FREE;
    atomicAdd(&A.qctl[2], 1);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// step kernels
// ---------------------------------------------------------------------------
// z for every listed slot (both lists): workgroups stride over the entries in
// x; gridDim.y workgroups share one slot's units (one, with the TSVD part, whose
// copy of y needs the whole slot)
__global__ void __launch_bounds__(KT) k_prep(EngineArgs A) {
  const int S = A.S;
  const int c64 = A.lists[2 * S], clo = A.lists[2 * S + 1];
  const int N = A.r * A.ld;
  for (int li = blockIdx.x; li < c64 + clo; li += gridDim.x) {
    const int s = li < c64 ? A.lists[li] : A.lists[S + (li - c64)];
    const int* sis = A.si + (long)s * SI_N;
    const int2 pj = phase_j(sis);
    const int ph = pj.x;
    double* zs = A.z + (long)s * A.NV;
    // a slot admitted in the last step: its preconditioner blocks, for the
    // units this thread applies them to below (k_claim_lists clears the flag)
    if (lazy_pinv(A) && sis[SI_PINV])
      build_pinv(A, s, blockIdx.y * blockDim.x, gridDim.y * blockDim.x);
    // source: the iterate u (residual step), v_j (Arnoldi) or a recycled u_rj
    if (ph == PH_ARNOLDI && A.vf32) {
      const float* srcf = A.Vf + ((long)s * (A.m + 1) + pj.y) * A.NV;
      if (A.use_precond) {
        dispatch_r(A.r, [&](auto R) {
          apply_pinv<decltype(R)::value>(A, s, srcf, zs, false, nullptr, blockIdx.y * blockDim.x,
                                         gridDim.y * blockDim.x);
        });
      } else {
        for (int e = blockIdx.y * blockDim.x + threadIdx.x; e < N; e += gridDim.y * blockDim.x)
          zs[e] = srcf[e];
      }
    } else {
    const double* src = ph == PH_RESTART ? A.x + (long)s * A.NV
                        : ph == PH_RECYC ? rec_u(A, s, sis[SI_BANK], sis[SI_RJ])
                                         : A.V + ((long)s * (A.m + 1) + pj.y) * A.NV;
    if (A.use_precond) {
      dispatch_r(A.r, [&](auto R) {
        apply_pinv<decltype(R)::value>(A, s, src, zs, false, nullptr, blockIdx.y * blockDim.x,
                                       gridDim.y * blockDim.x);
      });
    } else {
      for (int e = blockIdx.y * blockDim.x + threadIdx.x; e < N; e += gridDim.y * blockDim.x)
        zs[e] = src[e];
    }
    }
    if (A.pbar > 0) {
      __syncthreads();
      double* yc = A.Yc + (long)li * A.Ks;
      for (int e = threadIdx.x; e < N; e += blockDim.x) yc[e] = zs[e];
      __syncthreads();
    }
  }
}

// ---- low-rank part of the preconditioner (TSVD of the coupling) ----
// P = B - D Nt Mt^T with B the block-diagonal part; by SMW
//   P^-1 v = y + B^-1 D Nt Cp^-1 Mt^T y,  y = B^-1 v,  Cp = I - Mt^T B^-1 D Nt.
// Per step: k_prep (y), GEMM Tbuf = Yc Mt, k_cap (Sc = Cp^-1 Tbuf),
// GEMM Qc = Sc Nt^T, k_prep2 (z = y + B^-1 D Qc).
__global__ void __launch_bounds__(KT) k_cap(EngineArgs A, int ggrid) {
  __shared__ double t[kPbarMax];
  const int S = A.S, p = A.pbar;
  const int c64 = A.lists[2 * S], cnt = A.lists[2 * S + 2];
  const int mta = (cnt + kGemmBM - 1) / kGemmBM;
  const int KS = splitk_of(mta, 1, ggrid, A.Ks / 16);  // FP64 K-tile 16
  const long kstride = (long)mta * kGemmBM * 128;
  const double* src = KS > 1 ? A.Tpart : A.Tbuf;
  const int tid = threadIdx.x;
  for (int li = blockIdx.x; li < cnt; li += gridDim.x) {
    const int s = li < c64 ? A.lists[li] : A.lists[S + (li - c64)];
    __syncthreads();
    if (tid < p) {
      double v = 0;
      for (int k = 0; k < KS; ++k) v += src[k * kstride + (long)li * 128 + tid];
      t[tid] = v;
    }
    __syncthreads();
    if (tid < 128) {
      double v = 0;
      if (tid < p) {
        const double* ci = A.Cpinv + ((long)s * kPbarMax + tid) * kPbarMax;
        for (int i = 0; i < p; ++i) v += ci[i] * t[i];
      }
      A.Sc[(long)li * 128 + tid] = v;
    }
  }
}

__global__ void __launch_bounds__(KT) k_prep2(EngineArgs A) {
  const int S = A.S;
  const int c64 = A.lists[2 * S], cnt = A.lists[2 * S + 2];
  for (int li = blockIdx.x; li < cnt; li += gridDim.x) {
    const int s = li < c64 ? A.lists[li] : A.lists[S + (li - c64)];
    apply_pinv(A, s, A.Qc + (long)li * A.Ks, A.z + (long)s * A.NV, true, A.d + (long)s * A.r);
  }
}

// Admission part of the TSVD preconditioner: Cp = I - Mt^T B^-1 D Nt for the
// slot's new parameter (pbar x pbar, accumulated unit by unit through LDS,
// 4 x 4 register blocks per thread) and its inverse by Gauss-Jordan with
// partial pivoting.  A singular Cp leaves Cp^-1 = 0 (block-diagonal part only).
__global__ void __launch_bounds__(KT) k_capsetup(EngineArgs A) {
  constexpr int LW = 8;  // rho rows (unit x row a) per chunk
  __shared__ double Ml[LW * 2][kPbarMax];
  __shared__ double Wl[LW * 2][kPbarMax];
  __shared__ double Cm[kPbarMax][kPbarMax + 1];
  __shared__ double fcol[kPbarMax];
  __shared__ double dsh[kMaxRank];
  __shared__ int piv_sh, bad;
  const int s = blockIdx.x;
  int* si = A.si + (long)s * SI_N;
  if (si[SI_CAPSET] == 0) return;
  const int r = A.r, ld = A.ld, h = A.h, nu = A.n - h, p = A.pbar;
  const int tid = threadIdx.x;
  const int CH = max(1, LW / r);
  const int nb = (p + 3) / 4;
  const int jb = tid / nb, ib = tid % nb;
  const bool owner = tid < nb * nb;
  if (tid < r) dsh[tid] = A.d[(long)s * r + tid];
  if (tid == 0) bad = 0;
  const double* P = A.Pinv + (long)s * r * r * ld;
  double acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
  for (int u0 = 0; u0 < nu; u0 += CH) {
    const int cu = min(CH, nu - u0);
    __syncthreads();
    for (int e = tid; e < cu * r * kPbarMax; e += KT) {
      const int c = e % kPbarMax, ua = e / kPbarMax;
      const int a = ua % r, uu = ua / r;
      if (c >= p) {
        Ml[2 * ua][c] = Ml[2 * ua + 1][c] = Wl[2 * ua][c] = Wl[2 * ua + 1][c] = 0.0;
        continue;
      }
      bool pr;
      const int q = uslot(u0 + uu, h, pr);
      const long ea = (long)a * ld + q;
      Ml[2 * ua][c] = A.TsM[ea * 128 + c];
      Ml[2 * ua + 1][c] = pr ? A.TsM[(ea + 1) * 128 + c] : 0.0;
      double wr = 0, wi = 0;  // (B^-1 D Nt_c)[a] at this unit
      for (int b = 0; b < r; ++b) {
        const double* pb = P + (long)(a * r + b) * ld;
        const long eb = (long)b * ld + q;
        const double nr = dsh[b] * A.TsN[eb * 128 + c];
        if (pr) {
          const double ni = dsh[b] * A.TsN[(eb + 1) * 128 + c];
          wr += pb[q] * nr - pb[q + 1] * ni;
          wi += pb[q] * ni + pb[q + 1] * nr;
        } else {
          wr += pb[q] * nr;
        }
      }
      Wl[2 * ua][c] = wr;
      Wl[2 * ua + 1][c] = wi;
    }
    __syncthreads();
    if (owner) {
      for (int row = 0; row < 2 * cu * r; ++row) {
        double mv[4], wv[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          mv[x] = Ml[row][min(4 * jb + x, kPbarMax - 1)];
          wv[x] = Wl[row][min(4 * ib + x, kPbarMax - 1)];
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) acc[x][y] += mv[x] * wv[y];
      }
    }
  }
  __syncthreads();
  if (owner) {
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        const int j = 4 * jb + x, i = 4 * ib + y;
        if (j < p && i < p) Cm[j][i] = (i == j ? 1.0 : 0.0) - acc[x][y];
      }
  }
  // inverse into the slot's Cp^-1 (global), Gauss-Jordan on [Cm | Inv]
  double* Inv = A.Cpinv + (long)s * kPbarMax * kPbarMax;
  for (int e = tid; e < p * kPbarMax; e += KT) Inv[e] = (e / kPbarMax == e % kPbarMax) ? 1.0 : 0.0;
  __syncthreads();
  for (int c = 0; c < p; ++c) {
    if (tid == 0) {
      int pv = c;
      double best = fabs(Cm[c][c]);
      for (int i = c + 1; i < p; ++i)
        if (fabs(Cm[i][c]) > best) {
          best = fabs(Cm[i][c]);
          pv = i;
        }
      piv_sh = pv;
      if (!(best > 1e-13)) bad = 1;
    }
    __syncthreads();
    if (bad) break;
    const int pv = piv_sh;
    if (pv != c) {
      for (int k = tid; k < 2 * p; k += KT) {
        if (k < p) {
          const double t = Cm[c][k];
          Cm[c][k] = Cm[pv][k];
          Cm[pv][k] = t;
        } else {
          const int kk = k - p;
          const double t = Inv[c * kPbarMax + kk];
          Inv[c * kPbarMax + kk] = Inv[pv * kPbarMax + kk];
          Inv[pv * kPbarMax + kk] = t;
        }
      }
    }
    __syncthreads();
    const double inv = 1.0 / Cm[c][c];
    __syncthreads();
    for (int k = tid; k < 2 * p; k += KT) {
      if (k < p) Cm[c][k] *= inv;
      else Inv[c * kPbarMax + (k - p)] *= inv;
    }
    __syncthreads();
    if (tid < p) fcol[tid] = Cm[tid][c];
    __syncthreads();
    for (int e = tid; e < p * 2 * p; e += KT) {
      const int i = e / (2 * p), k = e % (2 * p);
      if (i == c) continue;
      const double f = fcol[i];
      if (k < p) Cm[i][k] -= f * Cm[c][k];
      else Inv[i * kPbarMax + (k - p)] -= f * Inv[c * kPbarMax + (k - p)];
    }
    __syncthreads();
  }
  if (bad)
    for (int e = tid; e < p * kPbarMax; e += KT) Inv[e] = 0.0;
  if (tid == 0) si[SI_CAPSET] = 0;
}

// X rows (li, a, b) = Vh_a o z_{slot(li), b} in precision T
template <class T> __device__ inline void put(T* X, long off, long plane, double v);
template <> __device__ inline void put<double>(double* X, long off, long, double v) { X[off] = v; }
template <> __device__ inline void put<float>(float* X, long off, long, double v) { X[off] = (float)v; }
template <> __device__ inline void put<__bf16>(__bf16* X, long off, long plane, double v) {
  const float f = (float)v;
  const __bf16 hi = (__bf16)f;
  X[off] = hi;
  X[off + plane] = (__bf16)(f - (float)hi);
}

// one unit u of X row li * r * r + a * r + b
template <class T>
__device__ inline void formx_unit(const EngineArgs& A, T* X, long plane, int which, int row,
                                  int u) {
  const int r = A.r, ld = A.ld;
  const int ab = row % (r * r), li = row / (r * r);
  const int a = ab / r, b = ab - a * r;
  const int s = A.lists[which * A.S + li];
  const double* va = A.Vh + (long)a * ld;
  const double* zb = A.z + (long)s * A.NV + (long)b * ld;
  const long base = (long)row * ld;
  bool pr;
  const int q = uslot(u, A.h, pr);
  if (pr) {
    const double ar = va[q], ai = va[q + 1], br = zb[q], bi = zb[q + 1];
    put<T>(X, base + q, plane, ar * br - ai * bi);
    put<T>(X, base + q + 1, plane, ar * bi + ai * br);
  } else {
    put<T>(X, base + q, plane, va[q] * zb[q]);
  }
}

template <class T>
__global__ void __launch_bounds__(KT) k_formX(EngineArgs A, T* X, long plane, int which) {
  const int r = A.r;
  const int cnt = A.lists[2 * A.S + which];
  const int nu = A.n - A.h;
  const long total = (long)cnt * r * r * nu;
  const long stride = (long)gridDim.x * blockDim.x;
  const long g0 = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (total + stride < 0x7fffffffL) {  // 32-bit index arithmetic (every practical size)
    for (int g = (int)g0; g < (int)total; g += (int)stride) {
      const int row = g / nu;
      formx_unit(A, X, plane, which, row, g - row * nu);
    }
  } else {
    for (long g = g0; g < total; g += stride) {
      const int row = (int)(g / nu);
      formx_unit(A, X, plane, which, row, (int)(g - (long)row * nu));
    }
  }
}

// w = z - D (sum_b z_b o K1_ab + sum_b Uh_b o H_(li,a,b)); H is the sum of
// the stream-K segments of the Cauchy GEMM (a launch of ggrid workgroups
// over gnk K-tiles), added in segment order.  One unit u of row li * r + a.
template <int RT, class HT>
__device__ inline void epilogue_unit(const EngineArgs& A, const HT* __restrict__ Hp,
                                     const SkPlan& plan, int bshift, long segstride, int which,
                                     int row, int u) {
  const int S = A.S, r = RT > 0 ? RT : A.r, ld = A.ld;
  const int li = row / r, a = row - li * r;
  const int s = A.lists[which * S + li];
  const double* zs = A.z + (long)s * A.NV;
  double* ws = A.w + (long)s * A.NV + (long)a * ld;
  const double da = A.d[(long)s * r + a];
  bool pr;
  const int q = uslot(u, A.h, pr);
  const int ct = q / kGemmBN;  // q and q + 1 share a column tile
  double sr = 0, si = 0;
  // segment range of GEMM row grow (sk_segments in 32-bit arithmetic: the
  // engine bounds t * nk below 2^31); the r rows of one (li, a) mostly share a
  // row tile, so it is worked out again only when the row tile changes
  int rt_seg = -1, s0 = 0, nseg = 0;
  auto segments = [&](int grow) {
    const int rt = grow >> bshift;
    if (rt != rt_seg) {
      const unsigned a0 = (unsigned)(ct * plan.mta + rt) * (unsigned)plan.nk;
      s0 = (int)(a0 / (unsigned)plan.per);
      nseg = (int)((a0 + (unsigned)plan.nk - 1u) / (unsigned)plan.per) - s0 + 1;
      rt_seg = rt;
    }
    return nseg;
  };
  // the r rows' contributions, added in b order
  auto add_row = [&](int b, double hr, double hi) {
    const double* k = A.K1 + (long)(a * r + b) * ld;
    const double* zb = zs + (long)b * ld;
    const double* ub = A.Uh + (long)b * ld;
    if (pr) {
      const double kr = k[q], ki = k[q + 1], zr = zb[q], zi = zb[q + 1];
      const double ur = ub[q], ui = ub[q + 1];
      sr += zr * kr - zi * ki + ur * hr - ui * hi;
      si += zr * ki + zi * kr + ur * hi + ui * hr;
    } else {
      sr += zb[q] * k[q] + ub[q] * hr;
    }
  };
  if constexpr (RT > 0) {
    // the partial sums of the r rows advance together, two segments at a
    // time, so the loads of all r rows are in flight at once (each row's sum
    // keeps segment order; a sweep's tail has up to 16 segments per tile)
    const HT* hb[RT];
    int ns[RT], nsmax = 0;
#pragma unroll
    for (int b = 0; b < RT; ++b) {
      const int grow = row * RT + b;  // GEMM row
      ns[b] = segments(grow);
      nsmax = ns[b] > nsmax ? ns[b] : nsmax;
      hb[b] = Hp + (long)grow * ld + q;
    }
    double hr[RT], hi[RT];
#pragma unroll
    for (int b = 0; b < RT; ++b) hr[b] = hi[b] = 0.0;
    for (int t = 0; t < nsmax; t += 2) {
      double vr[RT][2], vi[RT][2];
#pragma unroll
      for (int b = 0; b < RT; ++b)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const bool ok = t + e < ns[b];
          const HT* h = hb[b] + (t + e) * segstride;
          vr[b][e] = ok ? (double)h[0] : 0.0;
          vi[b][e] = ok && pr ? (double)h[1] : 0.0;
        }
#pragma unroll
      for (int b = 0; b < RT; ++b)
#pragma unroll
        for (int e = 0; e < 2; ++e)
          if (t + e < ns[b]) {
            hr[b] += vr[b][e];
            hi[b] += vi[b][e];
          }
    }
#pragma unroll
    for (int b = 0; b < RT; ++b) add_row(b, hr[b], hi[b]);
  } else {
    for (int b = 0; b < r; ++b) {
      const int grow = row * r + b;
      const int ns = segments(grow);
      const HT* hb = Hp + (long)grow * ld + q;
      // segments in order, two loads issued before their adds
      double hr = 0, hi = 0;
      int t = 0;
      for (; t + 2 <= ns; t += 2) {
        const HT* h0 = hb + t * segstride;
        const double r0 = (double)h0[0], r1 = (double)h0[segstride];
        const double i0 = pr ? (double)h0[1] : 0.0, i1 = pr ? (double)h0[segstride + 1] : 0.0;
        hr += r0;
        hr += r1;
        hi += i0;
        hi += i1;
      }
      if (t < ns) {
        hr += (double)hb[t * segstride];
        if (pr) hi += (double)hb[t * segstride + 1];
      }
      add_row(b, hr, hi);
    }
  }
  ws[q] = zs[(long)a * ld + q] - da * sr;
  if (pr) ws[q + 1] = zs[(long)a * ld + q + 1] - da * si;
}

template <class HT>
__global__ void __launch_bounds__(KT)
k_epilogue(EngineArgs A, const HT* Hp, int which, int ggrid, int gnk) {
  const int S = A.S, r = A.r, ld = A.ld;
  const int cnt = A.lists[2 * S + which];
  const int nu = A.n - A.h;
  const SkPlan plan = sk_plan(cnt * r * r, ld / kGemmBN, ggrid, gnk);
  const int bshift = plan.bm == 32 ? 5 : (plan.bm == 64 ? 6 : 7);
  const long segstride = (long)plan.mta * plan.bm * ld;
  const long total = (long)cnt * r * nu;
  const long stride = (long)gridDim.x * blockDim.x;
  const long g0 = (long)blockIdx.x * blockDim.x + threadIdx.x;
  dispatch_r(r, [&](auto R) {
    constexpr int RT = decltype(R)::value;
    if (total + stride < 0x7fffffffL) {  // 32-bit index arithmetic (every practical size)
      for (int g = (int)g0; g < (int)total; g += (int)stride) {
        const int row = g / nu;  // li * r + a
        epilogue_unit<RT>(A, Hp, plan, bshift, segstride, which, row, g - row * nu);
      }
    } else {
      for (long g = g0; g < total; g += stride) {
        const int row = (int)(g / nu);
        epilogue_unit<RT>(A, Hp, plan, bshift, segstride, which, row, (int)(g - (long)row * nu));
      }
    }
  });
}

// Schur basis: w = z - D out, out_s[a] = Vs_a^T Xs (projected seed solve)
// Dense Schur operator: rows of the listed slots' z (r ld values each) into
// consecutive rows of X, and the GEMM's rows back to the slots' rows of H.
__global__ void k_gather_z(EngineArgs A, double* __restrict__ X) {
  const int S = A.S;
  const int cnt = A.lists[2 * S];
  const long rl = (long)A.r * A.ld;
  for (int li = blockIdx.y; li < cnt; li += gridDim.y) {
    const int s = A.lists[li];
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < rl; e += (long)gridDim.x * blockDim.x)
      X[(long)li * rl + e] = A.z[(long)s * A.NV + e];
  }
}

__global__ void k_scatter_h(EngineArgs A, const double* __restrict__ Hc, double* __restrict__ H) {
  const int S = A.S;
  const int cnt = A.lists[2 * S];
  const long rl = (long)A.r * A.ld;
  for (int li = blockIdx.y; li < cnt; li += gridDim.y) {
    const int s = A.lists[li];
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < rl; e += (long)gridDim.x * blockDim.x)
      H[(long)s * rl + e] = Hc[(long)li * rl + e];
  }
}

__global__ void __launch_bounds__(KT) k_epilogue_schur(EngineArgs A, const double* out) {
  const int S = A.S, r = A.r, ld = A.ld;
  const int cnt = A.lists[2 * S];
  const int row = blockIdx.y;  // li * r + a
  const int li = row / r;
  if (li >= cnt) return;
  const int a = row % r;
  const int s = A.lists[li];
  const double da = A.d[(long)s * r + a];
  const double* zs = A.z + (long)s * A.NV + (long)a * ld;
  const double* os = out + ((long)s * r + a) * ld;
  double* ws = A.w + (long)s * A.NV + (long)a * ld;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < A.n; q += gridDim.x * blockDim.x)
    ws[q] = zs[q] - da * os[q];
}

// ---------------------------------------------------------------------------
// Krylov kernels.  One workgroup per slot; the slot's new vector w lives in
// registers as NE2 double2 per thread (element pair e2 = tid + KT * i of the
// padded slot vector, NV = 2 * KT * NE2), so each sweep over a basis streams
// every basis vector once with independent 16-byte loads, and all dot
// products of a pass are reduced with a single barrier.
// ---------------------------------------------------------------------------
constexpr int kPart = kMaxBasis + 2;
constexpr int kPartA = 2 * kMaxRestart + 2;  // a (m), b (m), c, d

// Orthogonalise w against the unit vectors vec(0..nvec-1): classical
// Gram-Schmidt, with a second pass only when the first one cancelled more
// than 1/sqrt(2) of ||w|| (Daniel-Gragg-Kaufman-Stewart criterion).
// coef[t] receives the summed projections; returns ||w|| afterwards and the
// norm before in wn0.
template <int NE2, int BT, class VecF>
__device__ double cgs2(double2 (&w2)[NE2], int nvec, VecF vec, double* coef,
                       double (*part)[kPart], double* ytmp, double* lds, double& wn0) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < nvec) coef[tid] = 0.0;
  double wn2 = 0.0, hn = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    double ww = 0.0;
    if (pass == 0) {
#pragma unroll
      for (int i = 0; i < NE2; ++i) ww += w2[i].x * w2[i].x + w2[i].y * w2[i].y;
    }
    int k = 0;
    for (; k + 4 <= nvec; k += 4) {
      double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
      const double2* v0 = reinterpret_cast<const double2*>(vec(k));
      const double2* v1 = reinterpret_cast<const double2*>(vec(k + 1));
      const double2* v2 = reinterpret_cast<const double2*>(vec(k + 2));
      const double2* v3 = reinterpret_cast<const double2*>(vec(k + 3));
#pragma unroll
      for (int i = 0; i < NE2; ++i) {
        const int e = tid + BT * i;
        const double2 x0 = v0[e], x1 = v1[e], x2 = v2[e], x3 = v3[e];
        a0 += x0.x * w2[i].x + x0.y * w2[i].y;
        a1 += x1.x * w2[i].x + x1.y * w2[i].y;
        a2 += x2.x * w2[i].x + x2.y * w2[i].y;
        a3 += x3.x * w2[i].x + x3.y * w2[i].y;
      }
      a0 = wave_sum(a0);
      a1 = wave_sum(a1);
      a2 = wave_sum(a2);
      a3 = wave_sum(a3);
      if (lane == 0) {
        part[wave][k] = a0;
        part[wave][k + 1] = a1;
        part[wave][k + 2] = a2;
        part[wave][k + 3] = a3;
      }
    }
    for (; k < nvec; ++k) {
      double a0 = 0;
      const double2* v0 = reinterpret_cast<const double2*>(vec(k));
#pragma unroll
      for (int i = 0; i < NE2; ++i) {
        const double2 x0 = v0[tid + BT * i];
        a0 += x0.x * w2[i].x + x0.y * w2[i].y;
      }
      a0 = wave_sum(a0);
      if (lane == 0) part[wave][k] = a0;
    }
    ww = wave_sum(ww);
    if (lane == 0) part[wave][kPart - 1] = ww;
    __syncthreads();
    if (tid < nvec) {
      double h = 0.0;
      for (int w = 0; w < BT / 64; ++w) h += part[w][tid];
      ytmp[tid] = h;
      coef[tid] += h;
    }
    if (pass == 0) {
      wn2 = 0.0;
      for (int w = 0; w < BT / 64; ++w) wn2 += part[w][kPart - 1];
      wn0 = sqrt(wn2);
    }
    __syncthreads();
    // w -= sum_k h_k v_k, four vectors per sweep step
    int kk = 0;
    for (; kk + 4 <= nvec; kk += 4) {
      const double c0 = ytmp[kk], c1 = ytmp[kk + 1], c2 = ytmp[kk + 2], c3 = ytmp[kk + 3];
      const double2* v0 = reinterpret_cast<const double2*>(vec(kk));
      const double2* v1 = reinterpret_cast<const double2*>(vec(kk + 1));
      const double2* v2 = reinterpret_cast<const double2*>(vec(kk + 2));
      const double2* v3 = reinterpret_cast<const double2*>(vec(kk + 3));
#pragma unroll
      for (int i = 0; i < NE2; ++i) {
        const int e = tid + BT * i;
        const double2 x0 = v0[e], x1 = v1[e], x2 = v2[e], x3 = v3[e];
        w2[i].x -= c0 * x0.x + c1 * x1.x + c2 * x2.x + c3 * x3.x;
        w2[i].y -= c0 * x0.y + c1 * x1.y + c2 * x2.y + c3 * x3.y;
      }
    }
    for (; kk < nvec; ++kk) {
      const double c = ytmp[kk];
      const double2* v0 = reinterpret_cast<const double2*>(vec(kk));
#pragma unroll
      for (int i = 0; i < NE2; ++i) {
        const double2 x0 = v0[tid + BT * i];
        w2[i].x -= c * x0.x;
        w2[i].y -= c * x0.y;
      }
    }
    double nn = 0.0;
#pragma unroll
    for (int i = 0; i < NE2; ++i) nn += w2[i].x * w2[i].x + w2[i].y * w2[i].y;
    nn = block_sum1(nn, lds);
    hn = sqrt(nn);
    if (!(nn < 0.5 * wn2)) break;  // no severe cancellation: one pass is enough
    wn2 = nn;
  }
  return hn;
}

// acc = sum_t coef[t] * vec(t) (registers)
template <int NE2, int BT, class VecF>
__device__ inline void combine(double2 (&acc)[NE2], int nvec, VecF vec, const double* coef) {
  for (int t = 0; t < nvec; ++t) {
    const double c = coef[t];
    const double2* v0 = reinterpret_cast<const double2*>(vec(t));
#pragma unroll
    for (int i = 0; i < NE2; ++i) {
      const double2 x0 = v0[threadIdx.x + BT * i];
      acc[i].x += c * x0.x;
      acc[i].y += c * x0.y;
    }
  }
}

template <int NE2, int BT = KT>
__device__ inline void store2(double* dst, const double2 (&v)[NE2], double scale) {
  double2* d2 = reinterpret_cast<double2*>(dst);
#pragma unroll
  for (int i = 0; i < NE2; ++i)
    d2[threadIdx.x + BT * i] = make_double2(v[i].x * scale, v[i].y * scale);
}

template <int NE2, int BT = KT>
__device__ inline void load2(double2 (&v)[NE2], const double* src) {
  const double2* s2 = reinterpret_cast<const double2*>(src);
#pragma unroll
  for (int i = 0; i < NE2; ++i) v[i] = s2[threadIdx.x + BT * i];
}

// u += U coef (current bank)
template <int NE2, int BT>
__device__ void x_add_recycled(const EngineArgs& A, int s, int bank, int nvec, const double* coef,
                               double2 (&tmp)[NE2]) {
  double* xs = A.x + (long)s * A.NV;
  load2<NE2, BT>(tmp, xs);
  combine<NE2, BT>(tmp, nvec, [&](int t) { return rec_u(A, s, bank, t); }, coef);
  store2<NE2, BT>(xs, tmp, 1.0);
}

// ---------------------------------------------------------------------------
// Split orthogonalisation of the Arnoldi step (restarted GMRES): classical
// Gram-Schmidt with one reorthogonalisation (CGS2).  A slot's vector is cut
// into chunks, one workgroup per slot and chunk (sizes below), so
// that the streaming of the basis V_0..j uses the whole chip also when few
// slots are active (one workgroup per slot leaves most CUs idle in a sweep's
// tail):
//   k_orth<0>  chunk partials of <v_k, w> (k <= j) and of ||w||^2        -> orth1
//   k_orth<1>  h = sum of those partials (fixed order), w -= V h on the
//              chunk; chunk partials of <v_k, w> and ||w||^2 again       -> orth1b
//   k_orth<2>  h' = sum of the second partials, w -= V h'; chunk partial
//              of ||w||^2                                                 -> orth2
// k_krylov sums the same partials in the same order (projections h + h',
// the norm), and runs a further single-workgroup pass only if the second one
// still cancelled more than half of ||w||^2.  With the block-diagonal
// preconditioner A P^-1 is close to the identity, so the first pass nearly
// always cancels most of w and the second pass is the rule, not the exception.
// ---------------------------------------------------------------------------
// Workgroups of OT threads take chunks of 2 OT values (one double2 per thread):
// 1024 threads (16 wavefronts, chunks of 2048) when the slot stride allows,
// 256 for the short vectors of small seeds.
inline int orth_threads(long long NV) { return NV % 2048 == 0 ? 1024 : 256; }

// part[wave][k] (k < nvec) and part[wave][kPart - 1] for one chunk, then the
// workgroup's sums to dst[0..nvec) and dst[kPart - 1]
template <int OT>
__device__ inline void chunk_dots(const double2 w, const double* V0, long NV, int nvec,
                                  double (*part)[kPart], double* dst) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  auto vk = [&](int k) { return reinterpret_cast<const double2*>(V0 + (long)k * NV)[tid]; };
  int k = 0;
  // eight vectors per step: all eight loads are issued before the reductions
  // (few slots in flight leave each workgroup latency-bound otherwise)
  for (; k + 8 <= nvec; k += 8) {
    double2 x[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = vk(k + q);
    double a[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = wave_sum(x[q].x * w.x + x[q].y * w.y);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 8; ++q) part[wave][k + q] = a[q];
    }
  }
  for (; k < nvec; ++k) {
    const double2 x0 = vk(k);
    const double a0 = wave_sum(x0.x * w.x + x0.y * w.y);
    if (lane == 0) part[wave][k] = a0;
  }
  const double ww = wave_sum(w.x * w.x + w.y * w.y);
  if (lane == 0) part[wave][kPart - 1] = ww;
  __syncthreads();
  for (int t = tid; t < nvec; t += OT) {
    double v = 0.0;
    for (int q = 0; q < OT / 64; ++q) v += part[q][t];
    dst[t] = v;
  }
  if (tid == 0) {
    double v = 0.0;
    for (int q = 0; q < OT / 64; ++q) v += part[q][kPart - 1];
    dst[kPart - 1] = v;
  }
  __syncthreads();
}

// w -= sum_k hs[k] v_k on one chunk
__device__ inline void chunk_update(double2& w, const double* V0, long NV, int nvec,
                                    const double* hs) {
  const int tid = threadIdx.x;
  auto vk = [&](int k) { return reinterpret_cast<const double2*>(V0 + (long)k * NV)[tid]; };
  int k = 0;
  for (; k + 8 <= nvec; k += 8) {
    double2 x[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = vk(k + q);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      w.x -= hs[k + q] * x[q].x;
      w.y -= hs[k + q] * x[q].y;
    }
  }
  for (; k < nvec; ++k) {
    const double2 x0 = vk(k);
    const double h0 = hs[k];
    w.x -= h0 * x0.x;
    w.y -= h0 * x0.y;
  }
}

// a chunk element pair of a basis vector stored as VT (double or float)
template <class VT> struct Pair2;
template <> struct Pair2<double> {
  typedef double2 type;
  __device__ static double2 load(const double* p, int i) { return reinterpret_cast<const double2*>(p)[i]; }
  __device__ static void store(double* p, int i, double2 v) { reinterpret_cast<double2*>(p)[i] = v; }
};
template <> struct Pair2<float> {
  typedef float2 type;
  __device__ static double2 load(const float* p, int i) {
    const float2 v = reinterpret_cast<const float2*>(p)[i];
    return make_double2(v.x, v.y);
  }
  __device__ static void store(float* p, int i, double2 v) {
    reinterpret_cast<float2*>(p)[i] = make_float2((float)v.x, (float)v.y);
  }
};
template <class VT> __device__ inline const VT* basis(const EngineArgs& A);
template <> __device__ inline const double* basis<double>(const EngineArgs& A) { return A.V; }
template <> __device__ inline const float* basis<float>(const EngineArgs& A) { return A.Vf; }

// Cycle end of restarted GMRES, split like the orthogonalisation: for every
// listed slot whose Arnoldi cycle ended in this step (SI_COMB = jn vectors),
// u += V y on each chunk, y stored by k_krylov in ycoefs.
template <int OT, class VT = double>
__global__ void __launch_bounds__(OT) k_combine(EngineArgs A) {
  constexpr int kChunk = 2 * OT;
  __shared__ double ys[kMaxRestart + 1];
  const int S = A.S, c64 = A.lists[2 * S], cnt = A.lists[2 * S + 2];
  const int c = blockIdx.y, tid = threadIdx.x;
  for (int li = blockIdx.x; li < cnt; li += gridDim.x) {
    const int s = li < c64 ? A.lists[li] : A.lists[S + (li - c64)];
    const int jn = A.si[(long)s * SI_N + SI_COMB];
    if (jn <= 0) continue;  // uniform over the workgroup
    for (int t = tid; t < jn; t += OT) ys[t] = A.ycoefs[(long)s * (kMaxRestart + 1) + t];
    __syncthreads();
    const long off = (long)c * kChunk;
    double2* xp = reinterpret_cast<double2*>(A.x + (long)s * A.NV + off) + tid;
    double2 x = *xp;
    // x += V y  is  x -= V (-y): the same streaming loop as the update
    for (int t = tid; t < jn; t += OT) ys[t] = -ys[t];
    __syncthreads();
    if (sizeof(VT) == 8) {
      chunk_update(x, A.V + (long)s * (A.m + 1) * A.NV + off, A.NV, jn, ys);
    } else {
      const VT* V0 = basis<VT>(A) + (long)s * (A.m + 1) * A.NV + off;
      int k = 0;
      for (; k + 8 <= jn; k += 8) {
        double2 v8[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v8[q] = Pair2<VT>::load(V0 + (long)(k + q) * A.NV, tid);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          x.x -= ys[k + q] * v8[q].x;
          x.y -= ys[k + q] * v8[q].y;
        }
      }
      for (; k < jn; ++k) {
        const double2 v0 = Pair2<VT>::load(V0 + (long)k * A.NV, tid);
        x.x -= ys[k] * v0.x;
        x.y -= ys[k] * v0.y;
      }
    }
    *xp = x;
    __syncthreads();  // ys is reused for the next slot
  }
}

template <int PASS, int OT>
__global__ void __launch_bounds__(OT) k_orth(EngineArgs A) {
  constexpr int kChunk = 2 * OT;
  __shared__ double part[OT / 64][kPart];
  __shared__ double hs[kMaxBasis + 1];
  const int S = A.S, c64 = A.lists[2 * S], cnt = A.lists[2 * S + 2];
  const int c = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int li = blockIdx.x; li < cnt; li += gridDim.x) {
    const int s = li < c64 ? A.lists[li] : A.lists[S + (li - c64)];
    const int* si = A.si + (long)s * SI_N;
    if (si[SI_PHASE] != PH_ARNOLDI) continue;  // uniform over the workgroup
    const int nvec = si[SI_J] + 1;
    const long off = (long)c * kChunk;
    double2* wp = reinterpret_cast<double2*>(A.w + (long)s * A.NV + off) + tid;
    double2 w = *wp;
    const double* V0 = A.V + (long)s * (A.m + 1) * A.NV + off;
    if (PASS > 0) {
      // projections of the previous pass, summed over the chunks in fixed order
      const double* prev = (PASS == 1 ? A.orth1 : A.orth1b) + (long)s * A.nchunk * kPart;
      for (int t = tid; t < nvec; t += OT)
        hs[t] = chunk_sum(A.nchunk, [&](int q) { return prev[(long)q * kPart + t]; });
      __syncthreads();
      chunk_update(w, V0, A.NV, nvec, hs);
      *wp = w;
    }
    if (PASS < 2) {
      double* dst = (PASS == 0 ? A.orth1 : A.orth1b) + ((long)s * A.nchunk + c) * kPart;
      chunk_dots<OT>(w, V0, A.NV, nvec, part, dst);
    } else {
      const double nn = wave_sum(w.x * w.x + w.y * w.y);
      if (lane == 0) part[wave][0] = nn;
      __syncthreads();
      if (tid == 0) {
        double v = 0.0;
        for (int q = 0; q < OT / 64; ++q) v += part[q][0];
        A.orth2[(long)s * A.nchunk + c] = v;
      }
      __syncthreads();  // part and hs are reused for the next slot
    }
  }
}

// ---------------------------------------------------------------------------
// Arnoldi with delayed reorthogonalisation (CGS2 with one projection pass per
// step; after Swirydowicz, Langou, Ananthan, Yang and Thomas, "Low
// synchronization Gram-Schmidt and GMRES algorithms", 2020, DCGS2).  At step
// j the basis holds q_0..q_{j-1} (orthonormal) and u_j, the next direction
// after ONE Gram-Schmidt pass, not normalised; the operator gave
// w = A P^-1 u_j.  One pass over [q_0..q_{j-1}, u_j, w] (k_orth_a) yields
//   a = Q^T u_j, b = Q^T w, c = u_j^T u_j, d = u_j^T w,
// from which k_krylov forms, without touching the vectors:
//   beta = sqrt(c - a^T a)           u_j = Q a + beta q_j (the second pass)
//   column j of H:  (A P^-1 q_j = (w - A P^-1 Q a) / beta, A P^-1 Q = Q H)
//     h_top = (b - (H a)_top) / beta,
//     h_jj  = ((d - a^T b) / beta - beta a_{j-1}) / beta,
//   and one update pass (k_orth_b) writes
//     q_j     = (u_j - Q a) / beta                      (into V_j)
//     u_{j+1} = (w - Q b) / beta - z q_j,  z = a_{j-1} + h_jj   (into V_{j+1})
//   with the chunk partials of ||u_{j+1}||^2, the subdiagonal h_{j+1,j}
//   (k_krylov_post: Givens rotation, convergence, cycle end).
// The basis is read twice per step instead of four times (classical CGS2 in
// three passes).  Column j-1 keeps h_{j,j-1} = ||u_j|| and its first-pass
// projections: the second pass changes them by O(eps ||w_{j-1}||), the size
// of the rounding already in the Arnoldi relation.
// ---------------------------------------------------------------------------
// Sum over the wavefront of eight values per lane (a butterfly that halves the
// values at each of the first three exchanges: 10 exchanges instead of 48).
// Lane L ends with the total of value 4 b5 + 2 b4 + b3 (the bits 5, 4, 3 of L);
// all eight lanes of its group hold it.  Fixed order: deterministic.
__device__ inline double wave_sum8(const double (&v)[8]) {
  const int lane = threadIdx.x & 63;
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
  double t4[4], t2[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double send = b5 ? v[i] : v[i + 4];
    t4[i] = (b5 ? v[i + 4] : v[i]) + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double send = b4 ? t4[i] : t4[i + 2];
    t2[i] = (b4 ? t4[i + 2] : t4[i]) + __shfl_xor(send, 16, 64);
  }
  const double send = b3 ? t2[0] : t2[1];
  double t = (b3 ? t2[1] : t2[0]) + __shfl_xor(send, 8, 64);
  t += __shfl_xor(t, 4, 64);
  t += __shfl_xor(t, 2, 64);
  t += __shfl_xor(t, 1, 64);
  return t;
}

template <int OT, class VT = double>
__global__ void __launch_bounds__(OT) k_orth_a(EngineArgs A) {
  constexpr int kChunk = 2 * OT;
  __shared__ double part[OT / 64][kPartA];
  const int S = A.S, c64 = A.lists[2 * S], cnt = A.lists[2 * S + 2];
  const int c = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = A.m;
  for (int li = blockIdx.x; li < cnt; li += gridDim.x) {
    const int s = li < c64 ? A.lists[li] : A.lists[S + (li - c64)];
    const int2 pj = phase_j(A.si + (long)s * SI_N);
    if (pj.x != PH_ARNOLDI) continue;  // uniform over the workgroup
    const int j = pj.y;
    const long off = (long)c * kChunk;
    const VT* V0 = basis<VT>(A) + (long)s * (m + 1) * A.NV + off;
    const double2 w = reinterpret_cast<const double2*>(A.w + (long)s * A.NV + off)[tid];
    const double2 u = Pair2<VT>::load(V0 + (long)j * A.NV, tid);
    auto vk = [&](int k) { return Pair2<VT>::load(V0 + (long)k * A.NV, tid); };
    // four basis vectors per group: <v, u> as values 0..3, <v, w> as 4..7
    const int grp = lane >> 3;  // the value this lane's group of eight ends with
    for (int k = 0; k < j; k += 4) {
      double2 x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = k + q < j ? vk(k + q) : make_double2(0.0, 0.0);
      double v[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        v[q] = x[q].x * u.x + x[q].y * u.y;
        v[4 + q] = x[q].x * w.x + x[q].y * w.y;
      }
      const double t = wave_sum8(v);
      if ((lane & 7) == 0 && k + (grp & 3) < j)
        part[wave][(grp < 4 ? 0 : m) + k + (grp & 3)] = t;
    }
    {
      double v[8] = {u.x * u.x + u.y * u.y, u.x * w.x + u.y * w.y, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      const double t = wave_sum8(v);
      if ((lane & 7) == 0 && grp < 2) part[wave][2 * m + grp] = t;
    }
    __syncthreads();
    double* dst = A.orthA + ((long)s * A.nchunk + c) * kPartA;
    for (int t = tid; t < 2 * m + 2; t += OT) {
      if (t < 2 * m && (t % m) >= j) continue;
      double v = 0.0;
      for (int q = 0; q < OT / 64; ++q) v += part[q][t];
      dst[t] = v;
    }
    __syncthreads();  // part is reused for the next slot
  }
}

// The update pass of the delayed reorthogonalisation (see k_orth_a): q_j into
// V_j, u_{j+1} into V_{j+1}, chunk partials of ||u_{j+1}||^2 -> orth2.
template <int OT, class VT = double>
__global__ void __launch_bounds__(OT) k_orth_b(EngineArgs A) {
  constexpr int kChunk = 2 * OT;
  __shared__ double cf[kPartA];
  __shared__ double part[OT / 64];
  const int S = A.S, c64 = A.lists[2 * S], cnt = A.lists[2 * S + 2];
  const int c = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = A.m;
  for (int li = blockIdx.x; li < cnt; li += gridDim.x) {
    const int s = li < c64 ? A.lists[li] : A.lists[S + (li - c64)];
    const int* si = A.si + (long)s * SI_N;
    const int passb = si[SI_PASSB], j = si[SI_J];  // both loads before the test
    if (!passb) continue;  // uniform over the workgroup
    const double* cb = A.coefB + (long)s * kPartA;
    for (int t = tid; t < 2 * m + 2; t += OT) cf[t] = cb[t];
    __syncthreads();
    const long off = (long)c * kChunk;
    VT* V0 = const_cast<VT*>(basis<VT>(A)) + (long)s * (m + 1) * A.NV + off;
    const double2 w = reinterpret_cast<const double2*>(A.w + (long)s * A.NV + off)[tid];
    const double2 u = Pair2<VT>::load(V0 + (long)j * A.NV, tid);
    double2 sa = make_double2(0.0, 0.0), sb = make_double2(0.0, 0.0);
    auto vk = [&](int k) { return Pair2<VT>::load(V0 + (long)k * A.NV, tid); };
    int k = 0;
    for (; k + 4 <= j; k += 4) {
      double2 x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = vk(k + q);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        sa.x += cf[k + q] * x[q].x;
        sa.y += cf[k + q] * x[q].y;
        sb.x += cf[m + k + q] * x[q].x;
        sb.y += cf[m + k + q] * x[q].y;
      }
    }
    for (; k < j; ++k) {
      const double2 x0 = vk(k);
      sa.x += cf[k] * x0.x;
      sa.y += cf[k] * x0.y;
      sb.x += cf[m + k] * x0.x;
      sb.y += cf[m + k] * x0.y;
    }
    const double ib = cf[2 * m], z = cf[2 * m + 1];
    double2 qv, un;
    qv.x = (u.x - sa.x) * ib;
    qv.y = (u.y - sa.y) * ib;
    un.x = (w.x - sb.x) * ib - z * qv.x;
    un.y = (w.y - sb.y) * ib - z * qv.y;
    Pair2<VT>::store(V0 + (long)j * A.NV, tid, qv);
    Pair2<VT>::store(V0 + (long)(j + 1) * A.NV, tid, un);
    const double nn = wave_sum(un.x * un.x + un.y * un.y);
    if (lane == 0) part[wave] = nn;
    __syncthreads();
    if (tid == 0) {
      double v = 0.0;
      for (int q = 0; q < OT / 64; ++q) v += part[q];
      A.orth2[(long)s * A.nchunk + c] = v;
    }
    __syncthreads();  // cf and part are reused for the next slot
  }
}

// Arnoldi step j of the delayed reorthogonalisation, after the update pass:
// h_{j+1,j} = ||u_{j+1}||, Givens rotation of column j, residual estimate,
// end of the cycle (back substitution, coefficients for k_combine).
__global__ void __launch_bounds__(64) k_krylov_post(EngineArgs A) {
  __shared__ double hcol[kMaxRestart + 2];
  __shared__ double cs_l[kMaxRestart], sn_l[kMaxRestart];
  __shared__ double Rl[kMaxRestart][kMaxRestart + 1];  // R[l][k]: column l, row k
  __shared__ double gl[kMaxRestart + 1];
  __shared__ int end_sh;
  const int s = blockIdx.x, tid = threadIdx.x;
  int* si = A.si + (long)s * SI_N;
  const int passb = si[SI_PASSB], j = si[SI_J];  // both loads before the test
  if (!passb) return;  // uniform over the workgroup
  const int m = A.m;
  const double* sdv = A.sdv + (long)s * SD_N;
  double* gs = A.g + (long)s * (m + 1);
  double* Rs = A.R + (long)s * m * (m + 1);
  double* css = A.cs + (long)s * m;
  double* sns = A.sn + (long)s * m;
  const double bn = sdv[SD_BNORM];
  const double* hu = A.Hu + ((long)s * m + j) * (m + 1);
  for (int k = tid; k <= j; k += 64) hcol[k] = hu[k];
  for (int k = tid; k < j; k += 64) {
    cs_l[k] = css[k];
    sn_l[k] = sns[k];
  }
  __syncthreads();
  if (tid == 0) {
    const double n2 = chunk_sum(A.nchunk, [&](int q) { return A.orth2[(long)s * A.nchunk + q]; });
    const double hn = sqrt(n2);
    hcol[j + 1] = hn;
    A.Hu[((long)s * m + j) * (m + 1) + j + 1] = hn;
    // the rotated entry k + 1 is carried in a register, so the loads of the
    // next rotation do not wait for the previous one
    double carry = hcol[0];
    for (int k = 0; k < j; ++k) {
      const double b = hcol[k + 1], c = cs_l[k], sk = sn_l[k];
      hcol[k] = c * carry + sk * b;
      carry = -sk * carry + c * b;
    }
    const double a = carry, b = hcol[j + 1];
    double cr, sg;
    if (b == 0.0) {
      cr = 1.0;
      sg = 0.0;
    } else {
      const double t = hypot(a, b);
      cr = a / t;
      sg = b / t;
    }
    css[j] = cr;
    sns[j] = sg;
    hcol[j] = cr * a + sg * b;
    const double gj = gs[j];
    gs[j] = cr * gj;
    gs[j + 1] = -sg * gj;
    const double est = fabs(gs[j + 1]);
    const int iters = si[SI_ITERS] + 1;
    si[SI_ITERS] = iters;
    si[SI_J] = j + 1;
    si[SI_PASSB] = 0;
    double target = 0.5 * A.tol * bn;
    if (A.mixed) target = fmax(target, A.inner_tol * sdv[SD_BETA]);
    end_sh = est <= target || j + 1 >= m || !(hn > 1e-300 * bn) || iters >= A.max_iter ||
             !isfinite(est);
  }
  __syncthreads();
  for (int k = tid; k <= j; k += 64) Rs[(long)j * (m + 1) + k] = hcol[k];
  if (!end_sh) return;  // uniform
  // end of the cycle: back substitution R y = g (R from columns 0..j), then
  // u += V y by k_combine
  const int jn = j + 1;
  // columns 0..j-1 (column j is in hcol)
  strided_map(j * jn, [&](int e) { const int l = e / jn; return Rs[(long)l * (m + 1) + (e - l * jn)]; },
              [&](int e, double v) { const int l = e / jn; Rl[l][e - l * jn] = v; });
  for (int k = tid; k < jn; k += 64) {
    Rl[j][k] = hcol[k];
    gl[k] = gs[k];
  }
  __syncthreads();
  // column-oriented back substitution over the wave: lane i keeps the
  // right-hand side entry i (jn <= 64 lanes) and subtracts column k's
  // contribution once y_k is known
  double v = tid < jn ? gl[tid] : 0.0, yv = 0.0;
  for (int k = jn - 1; k >= 0; --k) {
    const double yk = __shfl(v, k) / Rl[k][k];
    if (tid == k) yv = yk;
    if (tid < k) v -= Rl[k][tid] * yk;
  }
  if (tid < jn) A.ycoefs[(long)s * (kMaxRestart + 1) + tid] = yv;
  if (tid == 0) {
    si[SI_COMB] = jn;
    si[SI_PHASE] = PH_RESTART;
  }
}

// Per slot and step, according to the slot's phase:
//   RESTART  w = A P^-1 u: true residual r = D c0 - w, convergence test, finish or
//            start a new cycle (r projected off the recycle space C first)
//   ARNOLDI  w = A P^-1 v_j: orthogonalise against [C, V], Givens update;
//            at the cycle end u += V y - U B y
//   RECYC    w = A P^-1 u_rj for a recycled u (new parameter): C = A P^-1 U
//            rebuilt one column per step (incremental QR); then x0 from the
//            recycle space.
// With REC false the recycle space is empty and this is restarted GMRES.
template <int NE2, bool REC, int BT>
__global__ void __launch_bounds__(BT) k_krylov(EngineArgs A) {
  __shared__ double part[BT / 64][kPart];
  __shared__ double lds[(BT / 64) * 9];
  __shared__ double coef[kMaxBasis + 1];
  __shared__ double ytmp[kMaxBasis + 1];
  __shared__ double ycoef[kMaxRestart + 1];
  __shared__ double hcol[kMaxRestart + 2];
  __shared__ double tco[kMaxRecycle];
  __shared__ int next_phase;
  const int s = blockIdx.x;
  const int r = A.r, ld = A.ld, N = r * ld, NV = A.NV, m = A.m;
  int* si = A.si + (long)s * SI_N;
  double* sdv = A.sdv + (long)s * SD_N;
  const int2 pj = phase_j(si);
  const int ph = pj.x;
  if (ph != PH_ARNOLDI && ph != PH_RESTART && !(REC && ph == PH_RECYC)) return;

  double* Vs = A.V + (long)s * (m + 1) * NV;
  double* ws = A.w + (long)s * NV;
  double* gs = A.g + (long)s * (m + 1);
  double* Rs = A.R + (long)s * m * (m + 1);
  double* css = A.cs + (long)s * m;
  double* sns = A.sn + (long)s * m;
  const double bn = sdv[SD_BNORM];
  const int tid = threadIdx.x;
  const int kc = REC ? si[SI_KCUR] : 0;
  const int bank = REC ? si[SI_BANK] : 0;
  auto cvec = [&](int l) { return rec_c(A, s, bank, l); };
  const double* d = A.d + (long)s * r;

  double2 w2[NE2];
  if (REC || ph != PH_ARNOLDI || !A.dcgs) load2<NE2, BT>(w2, ws);
  double wn0 = 0.0;

  if (REC && ph == PH_RECYC) {
    // w = A P^-1 u_rj = sum_{l<rj} c_l rho_l + rho c_rj
    const int rj = si[SI_RJ];
    const double hn = cgs2<NE2, BT>(w2, rj, cvec, coef, part, ytmp, lds, wn0);
    const bool ok = isfinite(hn) && hn > 1e-10 * wn0;
    if (ok) {
      store2<NE2, BT>(rec_c(A, s, bank, rj), w2, 1.0 / hn);
      // u_rj = (u_rj - sum_l u_l rho_l) / rho keeps A P^-1 U = C
      double* urj = rec_u(A, s, bank, rj);
      load2<NE2, BT>(w2, urj);
      double2 acc[NE2];
#pragma unroll
      for (int i = 0; i < NE2; ++i) acc[i] = make_double2(0.0, 0.0);
      combine<NE2, BT>(acc, rj, [&](int t) { return rec_u(A, s, bank, t); }, coef);
#pragma unroll
      for (int i = 0; i < NE2; ++i) {
        w2[i].x -= acc[i].x;
        w2[i].y -= acc[i].y;
      }
      store2<NE2, BT>(urj, w2, 1.0 / hn);
    }
    const int kn = ok ? rj + 1 : rj;
    __syncthreads();
    if (!ok || kn == kc) {
      // C complete (or cut at a dependent column): u0 = U C^T b, b = D c0
      if (kn > 0) {
#pragma unroll
        for (int i = 0; i < NE2; ++i) {
          const int e = 2 * (tid + BT * i);
          w2[i].x = e < N ? d[e / ld] * A.c0[e] : 0.0;
          w2[i].y = e + 1 < N ? d[(e + 1) / ld] * A.c0[e + 1] : 0.0;
        }
        double dummy;
        cgs2<NE2, BT>(w2, kn, cvec, coef, part, ytmp, lds, dummy);
        x_add_recycled<NE2, BT>(A, s, bank, kn, coef, w2);
      }
      if (tid == 0) {
        si[SI_KCUR] = kn;
        si[SI_PHASE] = PH_RESTART;
      }
    } else if (tid == 0) {
      si[SI_RJ] = rj + 1;
    }
    if (tid == 0) si[SI_ITERS] += 1;
    return;
  }

  if (ph == PH_RESTART) {
    // w = A y ; residual r = D c0 - w into V0
    double acc = 0;
#pragma unroll
    for (int i = 0; i < NE2; ++i) {
      const int e = 2 * (tid + BT * i);
      const double r0 = e < N ? d[e / ld] * A.c0[e] - w2[i].x : 0.0;
      const double r1 = e + 1 < N ? d[(e + 1) / ld] * A.c0[e + 1] - w2[i].y : 0.0;
      w2[i].x = r0;
      w2[i].y = r1;
      acc += r0 * r0 + r1 * r1;
    }
    double rn = sqrt(block_sum1(acc, lds));
    const double rel = rn / bn;
    const int iters = si[SI_ITERS] + 1;
    const int refines = si[SI_REFINE];
    __syncthreads();
    if (tid == 0) si[SI_ITERS] = iters;
    __syncthreads();
    if (!isfinite(rel)) {
      finish(A, s, LYAP_E_NONFINITE, rel, lds);
    } else if (rel <= A.tol) {
      finish(A, s, LYAP_OK, rel, lds);
    } else if (iters >= A.max_iter || (A.mixed && refines >= A.max_refine)) {
      finish(A, s, LYAP_E_NOCONV, rel, lds);
    } else {
      if (REC && kc > 0) {
        // project r off C and add the matching correction U C^T r to u
        rn = cgs2<NE2, BT>(w2, kc, cvec, coef, part, ytmp, lds, wn0);
        if (rn > 0) store2<NE2, BT>(Vs, w2, 1.0 / rn);
        x_add_recycled<NE2, BT>(A, s, bank, kc, coef, w2);
        if (!(rn > 0)) {  // r lay in span(C): x is updated, test it again
          if (tid == 0) si[SI_PHASE] = PH_RESTART;
          return;
        }
      } else if (A.vf32) {
        float2* d2 = reinterpret_cast<float2*>(A.Vf + (long)s * (m + 1) * NV);
        const double sc = 1.0 / rn;
#pragma unroll
        for (int i = 0; i < NE2; ++i)
          d2[threadIdx.x + BT * i] = make_float2((float)(w2[i].x * sc), (float)(w2[i].y * sc));
      } else {
        store2<NE2, BT>(Vs, w2, 1.0 / rn);
      }
      if (tid == 0) {
        gs[0] = rn;
        sdv[SD_BETA] = rn;
        si[SI_J] = 0;
        si[SI_CYCLES] += 1;
        si[SI_REFINE] = refines + 1;
        si[SI_PHASE] = PH_ARNOLDI;
      }
      __syncthreads();
    }
    return;
  }

  // ---- Arnoldi step j: w = A P^-1 v_j, orthogonalised against [C, V_0..j] ----
  const int j = pj.y;  // the Arnoldi path does not write it before here
  if (!REC && A.dcgs) {
    // delayed reorthogonalisation (see k_orth_a): sums of the chunk partials,
    // beta, column j of H (unrotated, to Hu) and the update coefficients
    __shared__ double sa[kPartA];  // a (0..m-1), b (m..2m-1), c, d
    __shared__ double Hl[kMaxRestart][kMaxRestart + 1];  // H[k][i], k < j, i < j
    __shared__ double sbeta;
    double* cb = A.coefB + (long)s * kPartA;
    const double* pa = A.orthA + (long)s * A.nchunk * kPartA;
    for (int t = tid; t < 2 * m + 2; t += BT) {
      if (t < 2 * m && (t % m) >= j) continue;
      sa[t] = chunk_sum(A.nchunk, [&](int q) { return pa[(long)q * kPartA + t]; });
    }
    // the unrotated columns 0..j-1, rows 0..j-1
    const double* Hg = A.Hu + (long)s * m * (m + 1);
    strided_map(j * j, [&](int e) { const int k = e / j; return Hg[(long)k * (m + 1) + (e - k * j)]; },
                [&](int e, double v) { const int k = e / j; Hl[k][e - k * j] = v; });
    __syncthreads();
    // sum_k a_k^2 and sum_k a_k b_k over the first wave (j <= 64 terms)
    __shared__ double sab;
    if (tid < 64) {
      const double ak = tid < j ? sa[tid] : 0.0, bk = tid < j ? sa[m + tid] : 0.0;
      const double aa = wave_sum(ak * ak), ab = wave_sum(ak * bk);
      if (tid == 0) {
        const double cc = sa[2 * m];
        const double b2 = cc - aa;
        sbeta = b2 > 0.0 ? sqrt(b2) : sqrt(fmax(cc, 0.0));
        sab = ab;
      }
    }
    __syncthreads();
    const double beta = sbeta;
    double* hu = A.Hu + ((long)s * m + j) * (m + 1);
    // h_i = (b_i - (H a)_i) / beta for i < j; H upper Hessenberg (H[k][i] = 0 for i > k + 1)
    for (int i = tid; i < j; i += BT) {
      double v = 0.0;
      for (int k = (i > 0 ? i - 1 : 0); k < j; ++k) v += Hl[k][i] * sa[k];
      hu[i] = (sa[m + i] - v) / beta;
      cb[i] = sa[i];
      cb[m + i] = sa[m + i];
    }
    if (tid == 0) {
      const double ab = sab;
      const double dd = sa[2 * m + 1];
      const double ajm1 = j > 0 ? sa[j - 1] : 0.0;
      const double hjj = ((dd - ab) / beta - beta * ajm1) / beta;
      hu[j] = hjj;
      cb[2 * m] = 1.0 / beta;
      cb[2 * m + 1] = ajm1 + hjj;
      if (j == 0) gs[0] *= beta;  // r = ||r|| u_0 = ||r|| beta q_0
      si[SI_PASSB] = 1;
    }
    return;
  }
  double hn;
  if (REC) {
    hn = cgs2<NE2, BT>(
        w2, kc + j + 1,
        [&](int t) { return t < kc ? cvec(t) : Vs + (long)(t - kc) * NV; }, coef, part, ytmp, lds,
        wn0);
  } else {
    // two Gram-Schmidt passes done by k_orth<0..2> (w holds their result)
    __shared__ double norms[2];
    const double* p1 = A.orth1 + (long)s * A.nchunk * kPart;
    const double* p2 = A.orth1b + (long)s * A.nchunk * kPart;
    if (tid <= j) {
      const double a = chunk_sum(A.nchunk, [&](int q) { return p1[(long)q * kPart + tid]; });
      const double b = chunk_sum(A.nchunk, [&](int q) { return p2[(long)q * kPart + tid]; });
      coef[tid] = a + b;
    }
    if (tid == 0) {
      // ||w||^2 after the first pass and after the second
      norms[0] = chunk_sum(A.nchunk, [&](int q) { return p2[(long)q * kPart + kPart - 1]; });
      norms[1] = chunk_sum(A.nchunk, [&](int q) { return A.orth2[(long)s * A.nchunk + q]; });
    }
    __syncthreads();
    const double wn2 = norms[0], hn2 = norms[1];
    hn = sqrt(hn2);
    if (hn2 < 0.5 * wn2) {
      // the second pass cancelled again: a further pass in this workgroup
      load2<NE2, BT>(w2, ws);
      hn = cgs2<NE2, BT>(w2, j + 1, [&](int t) { return Vs + (long)t * NV; }, ycoef, part, ytmp,
                         lds, wn0);
      if (tid <= j) coef[tid] += ycoef[tid];
      __syncthreads();
    }
  }
  if (REC && tid < kc) A.Bk[((long)s * A.kmax + tid) * m + j] = coef[tid];
  if (tid <= j) hcol[tid] = coef[kc + tid];
  if (hn > 0) store2<NE2, BT>(Vs + (long)(j + 1) * NV, w2, 1.0 / hn);
  __syncthreads();
  if (tid == 0) {
    hcol[j + 1] = hn;
    if (REC) {
      double* hr = A.Hr + ((long)s * m + j) * (m + 1);
      for (int k = 0; k <= j + 1; ++k) hr[k] = hcol[k];
    }
    // apply previous rotations
    for (int k = 0; k < j; ++k) {
      const double a = hcol[k], b = hcol[k + 1];
      hcol[k] = css[k] * a + sns[k] * b;
      hcol[k + 1] = -sns[k] * a + css[k] * b;
    }
    const double a = hcol[j], b = hcol[j + 1];
    double c, sg;
    if (b == 0.0) {
      c = 1.0;
      sg = 0.0;
    } else {
      const double t = hypot(a, b);
      c = a / t;
      sg = b / t;
    }
    css[j] = c;
    sns[j] = sg;
    hcol[j] = c * a + sg * b;
    hcol[j + 1] = 0.0;
    for (int k = 0; k <= j; ++k) Rs[(long)j * (m + 1) + k] = hcol[k];
    const double gj = gs[j];
    gs[j] = c * gj;
    gs[j + 1] = -sg * gj;
    const double est = fabs(gs[j + 1]);
    const int iters = si[SI_ITERS] + 1;
    si[SI_ITERS] = iters;
    const int jn = j + 1;
    si[SI_J] = jn;
    double target = 0.5 * A.tol * bn;
    if (A.mixed) target = fmax(target, A.inner_tol * sdv[SD_BETA]);
    const bool end = est <= target || jn >= m || !(hn > 1e-300 * bn) || iters >= A.max_iter ||
                     !isfinite(est);
    // a new recycle space only where it can serve: the system restarts
    // unconverged, or queued parameters may still come to this slot
    const bool more = !(est <= 0.5 * A.tol * bn) ||
                      __atomic_load_n(&A.qctl[0], __ATOMIC_RELAXED) <
                          __atomic_load_n(&A.qctl[1], __ATOMIC_RELAXED);
    next_phase = !end ? PH_ARNOLDI : ((REC && A.kmax > 0 && more) ? PH_NEWSPACE : PH_RESTART);
    if (end) {
      // back substitution R y = g
      for (int k = jn - 1; k >= 0; --k) {
        double v = gs[k];
        for (int l = k + 1; l < jn; ++l) v -= Rs[(long)l * (m + 1) + k] * ycoef[l];
        ycoef[k] = v / Rs[(long)k * (m + 1) + k];
      }
      // recycle coefficients t = -B y (the C component of the minimiser)
      for (int l = 0; l < kc; ++l) {
        const double* bl = A.Bk + ((long)s * A.kmax + l) * m;
        double v = 0;
        for (int k = 0; k < jn; ++k) v += bl[k] * ycoef[k];
        tco[l] = -v;
      }
    }
  }
  __syncthreads();
  if (next_phase != PH_ARNOLDI) {
    const int jn = j + 1;
    // u += V y - U B y  (the iterate is kept before preconditioning)
    if (REC) {
      double* xs = A.x + (long)s * NV;
      load2<NE2, BT>(w2, xs);
      combine<NE2, BT>(w2, jn, [&](int t) { return Vs + (long)t * NV; }, ycoef);
      if (kc > 0) combine<NE2, BT>(w2, kc, [&](int t) { return rec_u(A, s, bank, t); }, tco);
      store2<NE2, BT>(xs, w2, 1.0);
    } else {
      // done by k_combine on all chunks after this kernel
      if (tid < jn) A.ycoefs[(long)s * (kMaxRestart + 1) + tid] = ycoef[tid];
      if (tid == 0) si[SI_COMB] = jn;
    }
    if (tid == 0) si[SI_PHASE] = next_phase;
  }
}

// ---------------------------------------------------------------------------
// Recycle-space update at the end of a cycle (GCRO-DR, deflated restart).
// The cycle gave  A P^-1 Vh = Wh G  with  Vh = [U Dk, V_0..mm-1],
// Wh = [C, V_0..mm]  (orthonormal),  G = [[Dk, B], [0, Hbar]]  (upper
// Hessenberg), Dk = diag(1/||u_l||).  Its Givens QR is G = Q R with
// Q = diag(I, Q_H), R = [[Dk, B], [0, R_H]].  Harmonic Ritz values theta of
// A P^-1 on span(Vh) are 1/mu for the eigenvalues mu of
// F = Q^T (Wh^T Vh) R^-1; the kt of smallest |theta| span the dominant
// invariant subspace Z of F (orthogonal iteration).  New space:
// U = Vh R^-1 Z,  C = Wh G R^-1 Z, orthonormalised together, so that
// A P^-1 U = C holds to the accuracy of the Arnoldi relation.
// ---------------------------------------------------------------------------
constexpr int kRecIters = 24;
constexpr int kRecScratch = (kMaxRestart + 1) * kMaxRestart;  // F, row-major, ld kMaxRestart

// in-place Cholesky of the kt x kt Gram matrix (thread 0); returns the number
// of leading columns that are numerically independent
__device__ inline int chol_small(double* Gm, int kt, int ldg) {
  double dmax = 0;
  for (int q = 0; q < kt; ++q) dmax = fmax(dmax, Gm[q * ldg + q]);
  for (int q = 0; q < kt; ++q) {
    double v = Gm[q * ldg + q];
    for (int p = 0; p < q; ++p) v -= Gm[q * ldg + p] * Gm[q * ldg + p];
    if (!(v > 1e-24 * dmax)) return q;
    const double lq = sqrt(v);
    Gm[q * ldg + q] = lq;
    for (int i = q + 1; i < kt; ++i) {
      double u = Gm[i * ldg + q];
      for (int p = 0; p < q; ++p) u -= Gm[i * ldg + p] * Gm[q * ldg + p];
      Gm[i * ldg + q] = u / lq;
    }
  }
  return kt;
}

template <int NE2>
__global__ void __launch_bounds__(KT) k_recycle(EngineArgs A) {
  constexpr int G = NE2 <= 8 ? 4 : (NE2 <= 16 ? 2 : 1);  // vectors held in registers
  constexpr int LDZ = kMaxRecycle;
  __shared__ double Z[kMaxRestart + 1][LDZ];
  __shared__ double FZ[kMaxRestart + 1][LDZ];
  __shared__ double CU[kMaxRecycle][kMaxRecycle];
  __shared__ double VU[kMaxRestart + 1][kMaxRecycle];
  __shared__ double part[4][(kMaxBasis + 1) * 4];
  __shared__ double Gm[kMaxRecycle * kMaxRecycle];
  __shared__ double dk[kMaxRecycle];
  __shared__ int kt_sh;
  const int s = blockIdx.x;
  int* si = A.si + (long)s * SI_N;
  if (si[SI_PHASE] != PH_NEWSPACE) return;
  const int m = A.m, NV = A.NV;
  const int kk = si[SI_KCUR], mm = si[SI_J], bank = si[SI_BANK];
  const int nh = kk + mm;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* Vs = A.V + (long)s * (m + 1) * NV;
  const double* Rs = A.R + (long)s * m * (m + 1);
  const double* Hr = A.Hr + (long)s * m * (m + 1);
  const double* Bk = A.Bk + (long)s * A.kmax * m;
  const double* css = A.cs + (long)s * m;
  const double* sns = A.sn + (long)s * m;
  double* F = A.Fs + (long)s * kRecScratch;
  auto wvec = [&](int t) { return t < kk ? rec_c(A, s, bank, t) : Vs + (long)(t - kk) * NV; };
  auto vvec = [&](int t) { return t < kk ? rec_u(A, s, bank, t) : Vs + (long)(t - kk) * NV; };

  // ---- A: dots  C^T U,  V_0..mm^T U  and ||u_l|| (G recycled vectors at a time) ----
  for (int l0 = 0; l0 < kk; l0 += G) {
    const int gn = min(G, kk - l0);
    double2 u[G][NE2];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (g < gn) load2<NE2>(u[g], rec_u(A, s, bank, l0 + g));
      else
#pragma unroll
        for (int i = 0; i < NE2; ++i) u[g][i] = make_double2(0.0, 0.0);
    }
    const int nt = kk + mm + 1;  // Wh columns
    for (int t = 0; t <= nt; ++t) {
      // t < nt: <Wh_t, u_g>;  t == nt: ||u_g||^2
      double a[G];
#pragma unroll
      for (int g = 0; g < G; ++g) a[g] = 0.0;
      if (t < nt) {
        const double2* x = reinterpret_cast<const double2*>(wvec(t));
#pragma unroll
        for (int i = 0; i < NE2; ++i) {
          const double2 xv = x[tid + KT * i];
#pragma unroll
          for (int g = 0; g < G; ++g) a[g] += xv.x * u[g][i].x + xv.y * u[g][i].y;
        }
      } else {
#pragma unroll
        for (int i = 0; i < NE2; ++i)
#pragma unroll
          for (int g = 0; g < G; ++g) a[g] += u[g][i].x * u[g][i].x + u[g][i].y * u[g][i].y;
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        a[g] = wave_sum(a[g]);
        if (lane == 0) part[wave][t * G + g] = a[g];
      }
    }
    __syncthreads();
    for (int e = tid; e < (nt + 1) * gn; e += KT) {
      const int t = e / gn, g = e % gn;
      const double v = part[0][t * G + g] + part[1][t * G + g] + part[2][t * G + g] +
                       part[3][t * G + g];
      const int l = l0 + g;
      if (t < kk) CU[t][l] = v;
      else if (t < nt) VU[t - kk][l] = v;
      else dk[l] = 1.0 / sqrt(v);
    }
    __syncthreads();
  }

  // R (nh x nh upper triangular) entry
  auto Rget = [&](int l, int c) -> double {
    if (l > c) return 0.0;
    if (c < kk) return l == c ? dk[c] : 0.0;
    const int cc = c - kk;
    return l < kk ? Bk[(long)l * m + cc] : Rs[(long)cc * (m + 1) + (l - kk)];
  };
  // G ((nh+1) x nh upper Hessenberg) entry
  auto Gget = [&](int i, int c) -> double {
    if (c < kk) return i == c ? dk[c] : 0.0;
    const int cc = c - kk;
    return i < kk ? Bk[(long)i * m + cc] : Hr[(long)cc * (m + 1) + (i - kk)];
  };

  // ---- B1: Y = Q^T (Wh^T Vh), one column per thread, into F ----
  if (tid < nh) {
    const int c = tid;
    // top rows (C^T): C^T U Dk for c < kk, 0 for the V columns
    for (int i = 0; i < kk; ++i) F[i * kMaxRestart + c] = c < kk ? CU[i][c] * dk[c] : 0.0;
    // bottom: Q_H^T applied to V^T U Dk or to e_(c-kk); rows kk..kk+mm of
    // column c serve as the work vector (row kk+mm is the spare row of F)
    double* col = F + (long)kk * kMaxRestart + c;
    for (int i = 0; i <= mm; ++i)
      col[i * kMaxRestart] = c < kk ? VU[i][c] * dk[c] : (i == c - kk ? 1.0 : 0.0);
    for (int i = 0; i < mm; ++i) {  // the cycle's rotations, in order
      const double a = col[i * kMaxRestart], b = col[(i + 1) * kMaxRestart];
      col[i * kMaxRestart] = css[i] * a + sns[i] * b;
      col[(i + 1) * kMaxRestart] = -sns[i] * a + css[i] * b;
    }
  }
  __syncthreads();
  // ---- B2: F = Y R^-1, one row per thread (forward substitution x R = y) ----
  if (tid < nh) {
    double* fr = F + tid * kMaxRestart;
    for (int c = 0; c < nh; ++c) {
      double v = fr[c];
      for (int l = 0; l < c; ++l) v -= fr[l] * Rget(l, c);
      fr[c] = v / Rget(c, c);
    }
  }
  if (tid == 0) kt_sh = min(A.kmax, nh);
  // deterministic start block
  for (int e = tid; e < nh * LDZ; e += KT) {
    const int i = e / LDZ, q = e % LDZ;
    unsigned h = (unsigned)(i * 2654435761u) ^ (unsigned)((q + 1) * 2246822519u);
    h ^= h >> 15;
    h *= 2654435761u;
    h ^= h >> 13;
    Z[i][q] = ((double)(h & 0xffffff) / 8388608.0) - 1.0;
  }
  __syncthreads();

  // ---- B3: orthogonal iteration on F, block orthonormalised by Cholesky QR ----
  for (int it = 0; it <= kRecIters; ++it) {
    const int kt = kt_sh;
    if (kt == 0) break;
    if (it > 0) {
      for (int e = tid; e < nh * kt; e += KT) {
        const int i = e / kt, q = e % kt;
        const double* fr = F + i * kMaxRestart;
        double v = 0;
        for (int l = 0; l < nh; ++l) v += fr[l] * Z[l][q];
        FZ[i][q] = v;
      }
    } else {
      for (int e = tid; e < nh * kt; e += KT) FZ[e / kt][e % kt] = Z[e / kt][e % kt];
    }
    __syncthreads();
    for (int e = tid; e < kt * kt; e += KT) {
      const int p = e / kt, q = e % kt;
      double v = 0;
      for (int i = 0; i < nh; ++i) v += FZ[i][p] * FZ[i][q];
      Gm[p * kMaxRecycle + q] = v;
    }
    __syncthreads();
    if (tid == 0) kt_sh = chol_small(Gm, kt, kMaxRecycle);
    __syncthreads();
    const int kn = kt_sh;
    // Z = FZ L^-T (row-wise), first kn columns
    if (tid < nh) {
      for (int q = 0; q < kn; ++q) {
        double v = FZ[tid][q];
        for (int p = 0; p < q; ++p) v -= Z[tid][p] * Gm[q * kMaxRecycle + p];
        Z[tid][q] = v / Gm[q * kMaxRecycle + q];
      }
    }
    __syncthreads();
  }
  const int kt = kt_sh;

  // ---- B4: P = R^-1 Z (in place, back substitution per column) ----
  if (tid < kt) {
    const int q = tid;
    for (int i = nh - 1; i >= 0; --i) {
      double v = Z[i][q];
      for (int l = i + 1; l < nh; ++l) v -= Rget(i, l) * Z[l][q];
      Z[i][q] = v / Rget(i, i);
    }
  }
  __syncthreads();
  // ---- B5: c = G P, then (c, P) L^-T twice so that Wh c is orthonormal ----
  int kf = kt;
  for (int rep = 0; rep < 3 && kf > 0; ++rep) {
    if (rep == 0) {
      for (int e = tid; e < (nh + 1) * kf; e += KT) {
        const int i = e / kf, q = e % kf;
        double v = 0;
        const int c0 = i < kk ? 0 : max(kk, kk + (i - kk) - 1);  // Hessenberg: G[i][c] = 0 for c < i-1
        for (int c = c0; c < nh; ++c) v += Gget(i, c) * Z[c][q];
        FZ[i][q] = v;
      }
      __syncthreads();
      continue;
    }
    for (int e = tid; e < kf * kf; e += KT) {
      const int p = e / kf, q = e % kf;
      double v = 0;
      for (int i = 0; i <= nh; ++i) v += FZ[i][p] * FZ[i][q];
      Gm[p * kMaxRecycle + q] = v;
    }
    __syncthreads();
    if (tid == 0) kt_sh = chol_small(Gm, kf, kMaxRecycle);
    __syncthreads();
    const int kn = kt_sh;
    if (tid <= nh) {
      for (int q = 0; q < kn; ++q) {
        double vc = FZ[tid][q], vp = tid < nh ? Z[tid][q] : 0.0;
        for (int p = 0; p < q; ++p) {
          vc -= FZ[tid][p] * Gm[q * kMaxRecycle + p];
          if (tid < nh) vp -= Z[tid][p] * Gm[q * kMaxRecycle + p];
        }
        FZ[tid][q] = vc / Gm[q * kMaxRecycle + q];
        if (tid < nh) Z[tid][q] = vp / Gm[q * kMaxRecycle + q];
      }
    }
    __syncthreads();
    kf = kn;
  }
  // fold Dk into the U rows of P; a non-finite coefficient drops the space
  for (int e = tid; e < kk * kf; e += KT) Z[e / kf][e % kf] *= dk[e / kf];
  if (tid == 0) kt_sh = 0;
  __syncthreads();
  for (int e = tid; e < (nh + 1) * kf; e += KT) {
    const int i = e / kf, q = e % kf;
    if (!isfinite(FZ[i][q]) || (i < nh && !isfinite(Z[i][q]))) kt_sh = 1;
  }
  __syncthreads();
  if (kt_sh) kf = 0;

  // ---- C: new U = Vh P, C = Wh c into the other bank ----
  const int nb = bank ^ 1;
  for (int q0 = 0; q0 < kf; q0 += G) {
    const int gn = min(G, kf - q0);
    for (int which = 0; which < 2; ++which) {
      double2 acc[G][NE2];
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int i = 0; i < NE2; ++i) acc[g][i] = make_double2(0.0, 0.0);
      const int nt = which == 0 ? nh : nh + 1;
      for (int t = 0; t < nt; ++t) {
        const double2* x = reinterpret_cast<const double2*>(which == 0 ? vvec(t) : wvec(t));
        double cf[G];
#pragma unroll
        for (int g = 0; g < G; ++g) cf[g] = g < gn ? (which == 0 ? Z[t][q0 + g] : FZ[t][q0 + g]) : 0.0;
#pragma unroll
        for (int i = 0; i < NE2; ++i) {
          const double2 xv = x[tid + KT * i];
#pragma unroll
          for (int g = 0; g < G; ++g) {
            acc[g][i].x += cf[g] * xv.x;
            acc[g][i].y += cf[g] * xv.y;
          }
        }
      }
#pragma unroll
      for (int g = 0; g < G; ++g)
        if (g < gn)
          store2<NE2>(which == 0 ? rec_u(A, s, nb, q0 + g) : rec_c(A, s, nb, q0 + g), acc[g], 1.0);
    }
  }
  __syncthreads();
  if (tid == 0) {
    si[SI_KCUR] = kf;
    si[SI_BANK] = nb;
    si[SI_PHASE] = PH_RESTART;
  }
}

// Per-slot vector stride.  Short vectors (r * ld <= 2048) use 256-thread
// Krylov workgroups and a stride of 512 * NE2 (NE2 = 1..4); longer ones use
// 1024 threads (16 wavefronts per slot) and a stride of 2048 * NE2 (NE2 =
// 2..8).  The recycle-update kernel runs 256 threads with stride / 512
// double2 per thread.
static long long slot_stride(long long r, long long ld) {
  const long long n = r * ld;
  if (n <= 2048) return 512LL * ((n + 511) / 512);
  const long long need = (n + 2 * KK - 1) / (2 * KK);
  LYAP_REQUIRE(need <= 8, LYAP_E_INVAL, "r * n too large for the Krylov kernel (r * ld <= 16384)");
  return 2LL * KK * need;
}

template <int NE2, int BT>
static void launch_krylov_ne(const EngineArgs& A, int S, hipStream_t st, bool update) {
  if (update) {
    hipLaunchKernelGGL((k_recycle<NE2 * BT / KT>), dim3(S), dim3(KT), 0, st, A);
  } else if (A.kmax > 0) {
    hipLaunchKernelGGL((k_krylov<NE2, true, BT>), dim3(S), dim3(BT), 0, st, A);
  } else {
    hipLaunchKernelGGL((k_krylov<NE2, false, BT>), dim3(S), dim3(BT), 0, st, A);
  }
}

// update selects the recycle-space update kernel instead of the Krylov step.
static void launch_krylov(const EngineArgs& A, int S, long long NV, hipStream_t st,
                          bool update = false) {
  if (NV <= 2048) {
    switch (NV / (2 * KT)) {
      case 1: launch_krylov_ne<1, KT>(A, S, st, update); return;
      case 2: launch_krylov_ne<2, KT>(A, S, st, update); return;
      case 3: launch_krylov_ne<3, KT>(A, S, st, update); return;
      case 4: launch_krylov_ne<4, KT>(A, S, st, update); return;
    }
  } else {
    switch (NV / (2 * KK)) {
      case 2: launch_krylov_ne<2, KK>(A, S, st, update); return;
      case 3: launch_krylov_ne<3, KK>(A, S, st, update); return;
      case 4: launch_krylov_ne<4, KK>(A, S, st, update); return;
      case 5: launch_krylov_ne<5, KK>(A, S, st, update); return;
      case 6: launch_krylov_ne<6, KK>(A, S, st, update); return;
      case 7: launch_krylov_ne<7, KK>(A, S, st, update); return;
      case 8: launch_krylov_ne<8, KK>(A, S, st, update); return;
    }
  }
  throw Error{LYAP_E_INVAL, "unsupported r * n for the Krylov kernel"};
}

// profiling: append this step's list counts at dst[2 * (*counter)]
// (graph-capturable: the position comes from a device counter)
__global__ void k_record_counts(const int* lists, int S, int* dst, int* counter) {
  const int i = counter[0];
  counter[0] = i + 1;
  dst[2 * i] = lists[2 * S];
  dst[2 * i + 1] = lists[2 * S + 1];
}

// Admission: every free slot takes the next queued parameter (device-side
// queue), so a slot freed in this step starts its next parameter in the next.
__global__ void __launch_bounds__(KT) k_admit(EngineArgs A) {
  __shared__ double lds[4 * 9];
  const int s = blockIdx.x;
  const int* si = A.si + (long)s * SI_N;
  if (si[SI_PHASE] != PH_FREE) return;  // uniform over the workgroup
  const int qp = si[SI_CLAIM];          // k_claim_lists
  if (qp >= 0) admit(A, s, qp, lds);
}

}  // namespace lyap

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
using namespace lyap;

// Launch configuration of the Cauchy GEMM chosen by the autotuner.
struct GemmTune {
  int bk = 0;               // K-tile depth (0: default)
  long long grid_min = 0;   // stream-K grid (workgroups)
  int xcd_off = 0;          // plain range order instead of the XCD-aware one
};

struct lyap_engine_s {
  lyap_seed sd = nullptr;
  GemmTune t64, tlo;  // Cauchy GEMM launch configurations (FP64, low precision)
  // workgroups of the grid-stride element kernels (k_formX, k_epilogue) and slot
  // workgroups per chunk of the orthogonalisation kernels (LYAP_EPI_GRID and
  // LYAP_ORTH_GRID override them for measurements)
  int egrid = 2048, og_cap = 1024;
  int S = 0, m = 40;
  lyap_solve_opts opts{};
  hipStream_t stream = nullptr;  // private non-blocking stream (graph capture needs one)
  bool mixed = false;
  GemmType low = GemmType::F64;
  int Q = 0;
  long long submitted = 0;   // queue positions handed out (host mirror of tail)
  long long harvested = 0;   // queue positions whose result was returned
  long long next_tag = 0;
  DevBuf si, sdv, d, R, g, cs, sn, V, x, z, w, Pinv, lists, X, H, Hp, Xlo, Hlo, Hplo, XS;
  DevBuf Ur, Cr, Bk, Hr, Fs;  // recycle space (GCRO-DR)
  DevBuf orth1, orth1b, orth2, ycoefs;  // split orthogonalisation (restarted GMRES)
  DevBuf orthA, coefB, Hu;              // its delayed-reorthogonalisation form
  DevBuf Vf;                            // FP32 basis of the low-precision modes
  DevBuf Cpinv, Tbuf, Tpart, Sc;  // low-rank preconditioner part
  DevBuf qd, qtag, qctl, res;
  double* sol = nullptr;
  long long sol_cap = 0;
  void* ws = nullptr;        // caller workspace the buffers are carved from (or null)
  bool owns_graph = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // profiling: captured step segments around the Cauchy products
  hipGraph_t pseg[3] = {nullptr, nullptr, nullptr};
  hipGraphExec_t psegx[3] = {nullptr, nullptr, nullptr};
  std::vector<hipEvent_t> pev;
  DevBuf pcounts;
  bool prof_graph_ok = true;
  bool prof_rec = false;  // while the profiled step segments are captured
  int prof_level = 0;        // level the profiling segments were captured with
  long long prof_step = 0;     // steps run while profiling (sampling)
  EngineArgs args{};
  std::vector<DevResult> res_host;
  std::vector<long long> done_pos;  // host-side list of positions already harvested
  std::vector<char> got;
  long long rows_pad = 0;
};

namespace lyap {

static void fill_defaults(lyap_solve_opts& o, const lyap_solve_opts* in) {
  o.prec = LYAP_PREC_FP64;
  o.max_iter = 600;
  o.restart = 64;
  o.use_precond = 1;
  o.recycle_k = 0;
  o.max_refine = 30;
  o.tol = 1e-12;
  o.inner_tol = 1e-4;
  if (!in) return;
  o.prec = in->prec;
  if (in->max_iter > 0) o.max_iter = in->max_iter;
  o.use_precond = in->use_precond;
  o.recycle_k = in->recycle_k;
  // default cycle: 64 for restarted GMRES, 40 with a recycle space (restart +
  // recycle_k <= 64)
  o.restart = in->restart > 0 ? in->restart : (o.recycle_k > 0 ? 40 : 64);
  if (in->max_refine > 0) o.max_refine = in->max_refine;
  if (in->tol > 0) o.tol = in->tol;
  if (in->inner_tol > 0) o.inner_tol = in->inner_tol;
}

// Arnoldi with delayed reorthogonalisation unless LYAP_ORTH=cgs2
static bool orth_dcgs() {
  const char* env = std::getenv("LYAP_ORTH");
  return !(env && std::string(env) == "cgs2");
}
// The Krylov basis of the low-precision modes is stored in FP32: their inner
// cycles only reduce the residual by inner_tol before an FP64 restart, so an
// FP32 basis (orthogonal to about 1e-7) halves the basis traffic at no cost in
// the refined result.  Restarted GMRES with the delayed reorthogonalisation
// only; LYAP_KRYLOV_F64=1 keeps FP64 (measurements).
static bool basis_f32(const lyap_solve_opts& o) {
  if (o.prec == LYAP_PREC_FP64 || o.recycle_k > 0 || !orth_dcgs()) return false;
  const char* env = std::getenv("LYAP_KRYLOV_F64");
  return !(env && std::string(env) == "1");
}

static void validate_opts(const lyap_solve_opts& o) {
  LYAP_REQUIRE(o.prec >= 0 && o.prec <= 3, LYAP_E_INVAL, "prec out of range");
  LYAP_REQUIRE(o.restart >= 1 && o.restart <= kMaxRestart, LYAP_E_INVAL, "restart out of [1, 64]");
  LYAP_REQUIRE(o.tol > 0 && o.tol < 1, LYAP_E_INVAL, "tol out of (0, 1)");
  LYAP_REQUIRE(o.max_iter >= 1, LYAP_E_INVAL, "max_iter < 1");
  LYAP_REQUIRE(o.use_precond >= 0 && o.use_precond <= 2, LYAP_E_INVAL, "use_precond out of [0, 2]");
  LYAP_REQUIRE(o.recycle_k >= 0 && o.recycle_k <= kMaxRecycle, LYAP_E_INVAL,
               "recycle_k out of [0, 16]");
  LYAP_REQUIRE(o.restart + o.recycle_k <= kMaxRestart, LYAP_E_INVAL,
               "restart + recycle_k > 64");
}

struct EngineSizes {
  size_t total = 0;
  long long rows_pad = 0;
};

// Every device buffer of an engine, in one fixed order: `take(buf, bytes)`
// with buf = nullptr when only sizes are wanted.  The engine's buffers come
// from its own allocations or are carved from a caller's workspace in this
// order, each rounded up to 256 bytes; engine_sizes is the same walk.
template <class F>
static void engine_layout(const lyap_seed_s* sd, long long S, const lyap_solve_opts& o, long long Q,
                          lyap_engine_s* E, F&& take) {
  const long long r = sd->r, ld = sd->ld, N = slot_stride(r, ld), m = o.restart;
  const long long rows_pad = pad_to(S * r * r, 128);
  auto t = [&](DevBuf lyap_engine_s::*mem, long long bytes) {
    take(E ? &(E->*mem) : nullptr, (size_t)bytes);
  };
  t(&lyap_engine_s::si, S * SI_N * 4);
  t(&lyap_engine_s::sdv, S * SD_N * 8);
  t(&lyap_engine_s::d, S * r * 8);
  t(&lyap_engine_s::R, S * m * (m + 1) * 8);
  t(&lyap_engine_s::g, S * (m + 1) * 8);
  t(&lyap_engine_s::cs, S * m * 8);
  t(&lyap_engine_s::sn, S * m * 8);
  const bool vf32 = basis_f32(o);
  t(&lyap_engine_s::V, vf32 ? 256 : S * (m + 1) * N * 8);
  t(&lyap_engine_s::Vf, vf32 ? S * (m + 1) * N * 4 : 256);
  t(&lyap_engine_s::x, S * N * 8);
  t(&lyap_engine_s::z, S * N * 8);
  t(&lyap_engine_s::w, S * N * 8);
  t(&lyap_engine_s::Pinv, S * r * r * ld * 8);
  t(&lyap_engine_s::lists, (2 * S + 3) * 4);
  const bool tsvd = sd->pbar > 0 && o.use_precond == 1 && r <= kPrecRank;
  if (tsvd) {
    const long long Sp = pad_to(S, 128);
    t(&lyap_engine_s::Cpinv, S * kPbarMax * kPbarMax * 8);
    t(&lyap_engine_s::Tbuf, Sp * 128 * 8);
    t(&lyap_engine_s::Sc, Sp * 128 * 8);
    t(&lyap_engine_s::Tpart, (long long)kTsvdGrid * 128 * 128 * 8);
  }
  if (o.recycle_k == 0) {
    const long long nch = N / (2 * orth_threads(N));
    t(&lyap_engine_s::orth1, S * nch * kPart * 8);
    t(&lyap_engine_s::orth1b, S * nch * kPart * 8);
    t(&lyap_engine_s::orth2, S * nch * 8);
    t(&lyap_engine_s::ycoefs, S * (kMaxRestart + 1) * 8);
    t(&lyap_engine_s::orthA, S * nch * kPartA * 8);
    t(&lyap_engine_s::coefB, S * kPartA * 8);
    t(&lyap_engine_s::Hu, S * m * (m + 1) * 8);
  }
  if (o.recycle_k > 0) {
    const long long k = o.recycle_k;
    t(&lyap_engine_s::Ur, S * 2 * k * N * 8);
    t(&lyap_engine_s::Cr, S * 2 * k * N * 8);
    t(&lyap_engine_s::Bk, S * k * m * 8);
    t(&lyap_engine_s::Hr, S * m * (m + 1) * 8);
    t(&lyap_engine_s::Fs, S * (long long)kRecScratch * 8);
  }
  if (sd->basis == LYAP_BASIS_SCHUR && !sd->Kd.p) t(&lyap_engine_s::XS, S * ld * ld * 8);
  t(&lyap_engine_s::X, rows_pad * ld * 8);
  t(&lyap_engine_s::H, rows_pad * ld * 8);
  t(&lyap_engine_s::Hp, cauchy_part_rows(rows_pad, ld, GemmType::F64) * ld * 8);
  if (o.prec != LYAP_PREC_FP64) {
    const GemmType lo = o.prec == LYAP_PREC_BF16_IR ? GemmType::BF16X3 : GemmType::F32;
    t(&lyap_engine_s::Xlo, rows_pad * ld * 4);
    t(&lyap_engine_s::Hlo, rows_pad * ld * 4);
    t(&lyap_engine_s::Hplo, cauchy_part_rows(rows_pad, ld, lo) * ld * 4);
  }
  t(&lyap_engine_s::qd, Q * r * 8);
  t(&lyap_engine_s::qtag, Q * 8);
  t(&lyap_engine_s::qctl, 16);
  t(&lyap_engine_s::res, Q * (long long)sizeof(DevResult));
}

static EngineSizes engine_sizes(const lyap_seed_s* sd, long long S, const lyap_solve_opts& o,
                                long long Q) {
  EngineSizes z;
  z.rows_pad = pad_to(S * sd->r * sd->r, 128);
  engine_layout(sd, S, o, Q, nullptr,
                [&](DevBuf*, size_t b) { z.total += (std::max<size_t>(b, 16) + 255) / 256 * 256; });
  return z;
}

// Optional event pairs around the kernels of one step (profiling mode).
struct StepEvents {
  hipEvent_t g64[2], glo[2], kry[2];
};

// Parts of one step: everything (PART_ALL), or the segments around the
// Cauchy products, so that a profiled step can replay the segments as graphs
// and launch the timed products between HIP events on the same stream.
enum StepPart { PART_ALL = -1, PART_PRE = 0, PART_G64 = 1, PART_MID = 2, PART_GLO = 3, PART_POST = 4 };

static void launch_step(lyap_engine_s* E, hipStream_t st, StepEvents* ev = nullptr,
                        int part = PART_ALL) {
  const EngineArgs& A = E->args;
  lyap_seed_s* sd = E->sd;
  const int S = E->S, r = (int)sd->r, ld = (int)sd->ld, nu = (int)(sd->n - sd->h);
  auto on = [&](int p) { return part == PART_ALL || part == p; };
  if (part != PART_ALL) ev = nullptr;
  const int pgrid = std::min(S, 1024);
  if (on(PART_PRE)) {
  {
    // units of one slot over several workgroups (full occupancy at full batch)
    const int pch = A.pbar > 0 ? 1 : std::max(1, std::min(16, (nu + KT - 1) / KT));
    hipLaunchKernelGGL(k_prep, dim3(pgrid, pch), dim3(KT), 0, st, A);
  }
  }
  if (on(PART_PRE) && A.pbar > 0) {
    // low-rank preconditioner part: two skinny GEMMs over the listed slots
    GemmArgs g{};
    g.type = GemmType::F64;
    g.A = A.Yc;
    g.B = A.TsM;
    g.C = A.Tbuf;
    g.M = S;
    g.N = 128;
    g.K = A.Ks;
    g.lda = A.Ks;
    g.ldb = g.ldc = g.Nstore = 128;
    g.M_dev = E->lists.as<int>() + 2 * S + 2;
    g.m_scale = 1;
    g.Cpart = A.Tpart;
    g.Cpart_rows = (long long)kTsvdGrid * 128;
    g.grid_min = kTsvdGrid;
    gemm_launch(g, st);
    const int ggrid = std::max((S + kGemmBM - 1) / kGemmBM, kTsvdGrid);
    hipLaunchKernelGGL(k_cap, dim3(pgrid), dim3(KT), 0, st, A, ggrid);
    GemmArgs q{};
    q.type = GemmType::F64;
    q.A = A.Sc;
    q.B = sd->TsNt.p;
    q.C = A.Qc;
    q.M = S;
    q.N = A.Ks;
    q.K = 128;
    q.lda = 128;
    q.ldb = q.ldc = q.Nstore = A.Ks;
    q.M_dev = E->lists.as<int>() + 2 * S + 2;
    q.m_scale = 1;
    gemm_launch(q, st);
    hipLaunchKernelGGL(k_prep2, dim3(pgrid), dim3(KT), 0, st, A);
  }
  const int ublocks = std::max(1, std::min((nu + KT - 1) / KT, 64));
  // grid-stride kernels: work proportional to the active count
  const int egrid = E->egrid;
  if (sd->basis == LYAP_BASIS_SCHUR && sd->Kd.p) {
    // dense capacitance operator: H rows of the listed slots = z rows Kd
    const long rl = (long)r * ld;
    const dim3 ggrid((unsigned)std::min<long>((rl + KT - 1) / KT, 16), (unsigned)std::min(S, 1024));
    if (on(PART_PRE))
    hipLaunchKernelGGL(k_gather_z, ggrid, dim3(KT), 0, st, A, E->X.as<double>());
    if (on(PART_G64)) {
    if (ev) LYAP_HIP(hipEventRecord(ev->g64[0], st));
    GemmArgs g{};
    g.type = GemmType::F64;
    g.A = E->X.p;
    g.B = sd->Kd.p;
    g.C = E->Hp.p;
    g.M = S;
    g.N = rl;
    g.K = rl;
    g.lda = g.ldb = g.ldc = rl;
    g.Nstore = rl;
    g.M_dev = E->lists.as<int>() + 2 * S;
    g.m_scale = 1;
    gemm_launch(g, st);
    if (ev) LYAP_HIP(hipEventRecord(ev->g64[1], st));
    }
    if (on(PART_MID)) {
    hipLaunchKernelGGL(k_scatter_h, ggrid, dim3(KT), 0, st, A, E->Hp.as<double>(),
                       E->H.as<double>());
    hipLaunchKernelGGL(k_epilogue_schur, dim3(ublocks, S * r), dim3(KT), 0, st, A,
                       E->H.as<double>());
    }
  } else if (sd->basis == LYAP_BASIS_SCHUR) {
    // seed solve in the real Schur basis for every listed slot
    const int n = (int)sd->n;
    const int* cnt = E->lists.as<int>() + 2 * S;
    if (on(PART_G64)) {
    if (ev) LYAP_HIP(hipEventRecord(ev->g64[0], st));
    trilyap_launch(sd->T.as<double>(), sd->Tt.as<double>(), E->XS.as<double>(), (long)ld * ld,
                   nullptr, 0, sd->Uh.as<double>(), E->z.as<double>(), (long)E->args.NV, r, n, ld, S,
                   E->lists.as<int>(), cnt, st);
    if (ev) LYAP_HIP(hipEventRecord(ev->g64[1], st));
    }
    if (on(PART_MID)) {
    project_launch(sd->Vh.as<double>(), E->XS.as<double>(), (long)ld * ld, E->H.as<double>(),
                   (long)r * ld, r, n, ld, S, E->lists.as<int>(), cnt, st);
    hipLaunchKernelGGL(k_epilogue_schur, dim3(ublocks, S * r), dim3(KT), 0, st, A,
                       E->H.as<double>());
    }
  } else {
  // FP64 list (which = 0)
  {
    if (on(PART_PRE))
    hipLaunchKernelGGL((k_formX<double>), dim3(egrid), dim3(KT), 0, st, A, E->X.as<double>(), 0L,
                       0);
    GemmArgs g{};
    g.type = GemmType::F64;
    g.A = E->X.p;
    g.B = sd->Mc.p;
    g.C = E->H.p;
    g.M = E->rows_pad;
    g.N = ld;
    g.K = ld;
    g.lda = g.ldb = g.ldc = ld;
    g.Nstore = ld;
    g.M_dev = E->lists.as<int>() + 2 * S;
    g.m_scale = r * r;
    g.Cpart = E->Hp.p;
    g.Cpart_rows = cauchy_part_rows(E->rows_pad, ld, GemmType::F64);
    g.bk = E->t64.bk;
    g.grid_min = E->t64.grid_min;
    g.xcd_off = E->t64.xcd_off;
    g.streamk = 1;
    if (on(PART_G64)) {
    if (ev) LYAP_HIP(hipEventRecord(ev->g64[0], st));
    gemm_launch(g, st);
    if (ev) LYAP_HIP(hipEventRecord(ev->g64[1], st));
    }
    if (on(PART_MID))
    hipLaunchKernelGGL((k_epilogue<double>), dim3(egrid), dim3(KT), 0, st, A, E->Hp.as<double>(),
                       0, (int)gemm_grid_of(g), gemm_nk_of(g));
  }
  if (E->mixed) {
    GemmArgs g{};
    g.B = (E->low == GemmType::F32) ? sd->Mc32.p : sd->Mcb.p;
    g.type = E->low;
    g.A = E->Xlo.p;
    g.C = E->Hlo.p;
    g.M = E->rows_pad;
    g.N = ld;
    g.K = ld;
    g.lda = g.ldb = g.ldc = ld;
    g.Nstore = ld;
    g.M_dev = E->lists.as<int>() + 2 * S + 1;
    g.m_scale = r * r;
    g.Cpart = E->Hplo.p;
    g.Cpart_rows = cauchy_part_rows(E->rows_pad, ld, E->low);
    g.bk = E->tlo.bk;
    g.grid_min = E->tlo.grid_min;
    g.xcd_off = E->tlo.xcd_off;
    g.streamk = 1;
    if (E->low != GemmType::F32) {
      g.a_plane = E->rows_pad * ld;
      g.b_plane = (long long)ld * ld;
    }
    if (on(PART_MID)) {
      if (E->low == GemmType::F32)
        hipLaunchKernelGGL((k_formX<float>), dim3(egrid), dim3(KT), 0, st, A, E->Xlo.as<float>(),
                           0L, 1);
      else
        hipLaunchKernelGGL((k_formX<__bf16>), dim3(egrid), dim3(KT), 0, st, A,
                           E->Xlo.as<__bf16>(), (long)(E->rows_pad * ld), 1);
    }
    if (on(PART_GLO)) {
    if (ev) LYAP_HIP(hipEventRecord(ev->glo[0], st));
    gemm_launch(g, st);
    if (ev) LYAP_HIP(hipEventRecord(ev->glo[1], st));
    }
    if (on(PART_POST))
    hipLaunchKernelGGL((k_epilogue<float>), dim3(egrid), dim3(KT), 0, st, A,
                       E->Hplo.as<float>(), 1, (int)gemm_grid_of(g), gemm_nk_of(g));
  }
  }  // eigen basis
  if (!on(PART_POST)) {
    LYAP_HIP(hipGetLastError());
    return;
  }
  if (ev && ev->kry[0]) LYAP_HIP(hipEventRecord(ev->kry[0], st));
  const int og = std::min(S, E->og_cap);
  const bool big = orth_threads(A.NV) == 1024;
  if (A.kmax == 0 && A.dcgs) {
    // delayed reorthogonalisation: projections, coefficients, update, Givens
    const dim3 og2(og, A.nchunk);
    if (A.vf32) {
      if (big)
        hipLaunchKernelGGL((k_orth_a<1024, float>), og2, dim3(1024), 0, st, A);
      else
        hipLaunchKernelGGL((k_orth_a<256, float>), og2, dim3(256), 0, st, A);
    } else {
      if (big)
        hipLaunchKernelGGL((k_orth_a<1024>), og2, dim3(1024), 0, st, A);
      else
        hipLaunchKernelGGL((k_orth_a<256>), og2, dim3(256), 0, st, A);
    }
    launch_krylov(A, S, (long long)A.NV, st);
    if (A.vf32) {
      if (big)
        hipLaunchKernelGGL((k_orth_b<1024, float>), og2, dim3(1024), 0, st, A);
      else
        hipLaunchKernelGGL((k_orth_b<256, float>), og2, dim3(256), 0, st, A);
    } else {
      if (big)
        hipLaunchKernelGGL((k_orth_b<1024>), og2, dim3(1024), 0, st, A);
      else
        hipLaunchKernelGGL((k_orth_b<256>), og2, dim3(256), 0, st, A);
    }
    hipLaunchKernelGGL(k_krylov_post, dim3(S), dim3(64), 0, st, A);
  } else {
    if (A.kmax == 0) {
      if (big) {
        hipLaunchKernelGGL((k_orth<0, 1024>), dim3(og, A.nchunk), dim3(1024), 0, st, A);
        hipLaunchKernelGGL((k_orth<1, 1024>), dim3(og, A.nchunk), dim3(1024), 0, st, A);
        hipLaunchKernelGGL((k_orth<2, 1024>), dim3(og, A.nchunk), dim3(1024), 0, st, A);
      } else {
        hipLaunchKernelGGL((k_orth<0, 256>), dim3(og, A.nchunk), dim3(256), 0, st, A);
        hipLaunchKernelGGL((k_orth<1, 256>), dim3(og, A.nchunk), dim3(256), 0, st, A);
        hipLaunchKernelGGL((k_orth<2, 256>), dim3(og, A.nchunk), dim3(256), 0, st, A);
      }
    }
    launch_krylov(A, S, (long long)A.NV, st);
  }
  if (A.kmax == 0) {
    const bool big = orth_threads(A.NV) == 1024;
    if (A.vf32) {
      if (big)
        hipLaunchKernelGGL((k_combine<1024, float>), dim3(og, A.nchunk), dim3(1024), 0, st, A);
      else
        hipLaunchKernelGGL((k_combine<256, float>), dim3(og, A.nchunk), dim3(256), 0, st, A);
    } else {
      if (big)
        hipLaunchKernelGGL((k_combine<1024>), dim3(og, A.nchunk), dim3(1024), 0, st, A);
      else
        hipLaunchKernelGGL((k_combine<256>), dim3(og, A.nchunk), dim3(256), 0, st, A);
    }
  }
  if (ev && ev->kry[0]) LYAP_HIP(hipEventRecord(ev->kry[1], st));
  if (A.kmax > 0) launch_krylov(A, S, (long long)A.NV, st, true);
  if (E->prof_rec)  // profiled steps: this step's list counts, before the next step's
    hipLaunchKernelGGL(k_record_counts, dim3(1), dim3(1), 0, st, E->lists.as<int>(), E->S,
                       E->pcounts.as<int>() + 1, E->pcounts.as<int>());
  hipLaunchKernelGGL(k_claim_lists, dim3(1), dim3(1024), 0, st, A);
  hipLaunchKernelGGL(k_admit, dim3(S), dim3(KT), 0, st, A);
  if (A.use_precond && !lazy_pinv(A))  // else the next step's k_prep builds the blocks
    hipLaunchKernelGGL(k_pinv, dim3(S, pinv_chunks(r, nu)), dim3(KT), 0, st, A);
  if (A.pbar > 0) hipLaunchKernelGGL(k_capsetup, dim3(S), dim3(KT), 0, st, A);
  LYAP_HIP(hipGetLastError());
}

// ---- process-wide profile (lyap_profile_*) ----
namespace {
std::mutex g_prof_mu;
int g_prof_level = 0;  // 0 off, 1 Cauchy GEMM events, 2 also the Krylov kernel
lyap_profile g_prof{};
}  // namespace

static int profiling() {
  std::lock_guard<std::mutex> g(g_prof_mu);
  return g_prof_level;
}

constexpr int kProfSteps = 8;
constexpr int kProfEvery = 4;

static void prof_accumulate(lyap_engine_s* E, const std::vector<StepEvents>& evs, const int* counts,
                            long long k, bool graph) {
  const double r = (double)E->sd->r, n = (double)E->sd->n;
  lyap_profile add{};
  for (long long i = 0; i < k; ++i) {
    float t = 0;
    LYAP_HIP(hipEventElapsedTime(&t, evs[i].g64[0], evs[i].g64[1]));
    if (counts[2 * i] > 0) {
      add.gemm64_ms += t;
      add.gemm64_launches += 1;
      add.gemm64_flops += 2.0 * counts[2 * i] * r * r * n * n;
    }
    if (E->mixed) {
      LYAP_HIP(hipEventElapsedTime(&t, evs[i].glo[0], evs[i].glo[1]));
      if (counts[2 * i + 1] > 0) {
        add.gemmlo_ms += t;
        add.gemmlo_launches += 1;
        add.gemmlo_flops += 2.0 * counts[2 * i + 1] * r * r * n * n;
      }
    }
    if (evs[i].kry[0]) {
      LYAP_HIP(hipEventElapsedTime(&t, evs[i].kry[0], evs[i].kry[1]));
      add.krylov_ms += t;
      add.krylov_launches += 1;
    }
    add.slot_steps += counts[2 * i] + counts[2 * i + 1];
  }
  add.steps = k;
  add.graph_steps = graph ? k : 0;
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof.graph_steps += add.graph_steps;
  g_prof.gemm64_ms += add.gemm64_ms;
  g_prof.gemm64_launches += add.gemm64_launches;
  g_prof.gemm64_flops += add.gemm64_flops;
  g_prof.gemmlo_ms += add.gemmlo_ms;
  g_prof.gemmlo_launches += add.gemmlo_launches;
  g_prof.gemmlo_flops += add.gemmlo_flops;
  g_prof.krylov_ms += add.krylov_ms;
  g_prof.krylov_launches += add.krylov_launches;
  g_prof.slot_steps += add.slot_steps;
  g_prof.steps += add.steps;
}

static std::vector<StepEvents> prof_events(lyap_engine_s* E) {
  std::vector<StepEvents> evs(kProfSteps);
  for (int i = 0; i < kProfSteps; ++i) {
    hipEvent_t* p = &evs[i].g64[0];
    for (int q = 0; q < 6; ++q) p[q] = E->pev[6 * i + q];
    if (E->prof_level < 2) evs[i].kry[0] = evs[i].kry[1] = nullptr;  // GEMM events only
  }
  return evs;
}

// Profiled steps.  Event-record nodes inside a graph cannot be read back
// with hipEventElapsedTime on this runtime, so a profiled step replays three
// captured segments (before, between and after the Cauchy products) and
// launches the products themselves directly, each between two HIP events on
// the engine stream; per-step active counts are appended by a small kernel
// in the last segment.  Level 2 (also timing the Krylov kernel) and any
// failure fall back to direct launches of whole steps.
static void prof_segments_build(lyap_engine_s* E) {
  hipStream_t st = E->stream;
  if (E->pev.empty()) {
    E->pev.resize(6 * kProfSteps);
    for (auto& e : E->pev) LYAP_HIP(hipEventCreate(&e));
    E->pcounts.alloc(sizeof(int) * (2 * kProfSteps + 1));
  }
  const int parts[3] = {PART_PRE, PART_MID, PART_POST};
  for (int q = 0; q < 3; ++q) {
    LYAP_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
      E->prof_rec = parts[q] == PART_POST;  // counts recorded inside the step
      launch_step(E, st, nullptr, parts[q]);
      E->prof_rec = false;
    } catch (...) {
      E->prof_rec = false;
      hipGraph_t tmp;
      (void)hipStreamEndCapture(st, &tmp);
      throw;
    }
    LYAP_HIP(hipStreamEndCapture(st, &E->pseg[q]));
    LYAP_HIP(hipGraphInstantiate(&E->psegx[q], E->pseg[q], nullptr, nullptr, 0));
  }
}

// Run k steps with event pairs around the Cauchy products and per-step active
// counts; accumulate the profile.
static void profiled_steps(lyap_engine_s* E, long long k, int level) {
  hipStream_t st = E->stream;
  const int S = E->S;
  if (level == 1 && E->prof_graph_ok) {
    try {
      if (!E->psegx[0]) prof_segments_build(E);
      E->prof_level = level;
      std::vector<StepEvents> evs = prof_events(E);
      int counts[2 * kProfSteps];
      for (long long done = 0; done < k; done += kProfSteps) {
        const int kk = (int)std::min<long long>(kProfSteps, k - done);
        LYAP_HIP(hipMemsetAsync(E->pcounts.p, 0, sizeof(int), st));
        int timed = 0;
        for (int j = 0; j < kk; ++j) {
          // time every kProfEvery-th step of the engine's life (uniform over
          // full-batch and tail steps); the others replay the production graph
          if (E->prof_step++ % kProfEvery != 0) {
            if (E->gexec) LYAP_HIP(hipGraphLaunch(E->gexec, st));
            else launch_step(E, st);
            continue;
          }
          const int i = timed++;
          LYAP_HIP(hipGraphLaunch(E->psegx[0], st));
          LYAP_HIP(hipEventRecord(evs[i].g64[0], st));
          launch_step(E, st, nullptr, PART_G64);
          LYAP_HIP(hipEventRecord(evs[i].g64[1], st));
          LYAP_HIP(hipGraphLaunch(E->psegx[1], st));
          if (E->mixed) {
            LYAP_HIP(hipEventRecord(evs[i].glo[0], st));
            launch_step(E, st, nullptr, PART_GLO);
            LYAP_HIP(hipEventRecord(evs[i].glo[1], st));
          }
          LYAP_HIP(hipGraphLaunch(E->psegx[2], st));
        }
        if (timed > 0) {
          LYAP_HIP(hipMemcpyAsync(counts, E->pcounts.as<int>() + 1, sizeof(int) * 2 * timed,
                                  hipMemcpyDeviceToHost, st));
          LYAP_HIP(hipStreamSynchronize(st));
          prof_accumulate(E, evs, counts, timed, true);
        }
      }
      return;
    } catch (const Error& e) {
      E->prof_graph_ok = false;
      (void)hipGetLastError();
      set_last_error("profiling segments unavailable, direct launches: " + e.msg);
    }
  }
  std::vector<StepEvents> evs(k);
  for (auto& e : evs)
    for (hipEvent_t* p : {&e.g64[0], &e.g64[1], &e.glo[0], &e.glo[1], &e.kry[0], &e.kry[1]})
      LYAP_HIP(hipEventCreate(p));
  int* counts = nullptr;
  LYAP_HIP(hipHostMalloc((void**)&counts, sizeof(int) * 2 * k, hipHostMallocDefault));
  for (long long i = 0; i < k; ++i) {
    // the lists of step i were built at the end of the step before it
    LYAP_HIP(hipMemcpyAsync(counts + 2 * i, E->lists.as<int>() + 2 * S, 2 * sizeof(int),
                            hipMemcpyDeviceToHost, st));
    launch_step(E, st, &evs[i]);
  }
  LYAP_HIP(hipStreamSynchronize(st));
  prof_accumulate(E, evs, counts, k, false);
  (void)hipHostFree(counts);
  for (auto& e : evs)
    for (hipEvent_t p : {e.g64[0], e.g64[1], e.glo[0], e.glo[1], e.kry[0], e.kry[1]})
      (void)hipEventDestroy(p);
}

// ---- launch autotuner of the Cauchy GEMM ----
// The Cauchy GEMMs run stream-K.  For the engine's GEMM shape (rows_pad x ld
// x ld) every candidate launch configuration (K-tile depth x grid of 2 or 4
// workgroups per CU x range order) is timed with HIP events at three
// active-row counts that stand for a sweep: the full batch, an eighth of it
// and 32 rows (the tail), weighted by the share of steps spent in each
// (0.15, 0.15, 0.7); each figure is the median of 5 timings of 2 launches.
// A candidate replaces the default launch (K-tile 16/32, two workgroups per
// CU, plain range order) only when it is more than 3% faster, so that timing
// noise does not flip the choice.  The result is kept for the process, per
// (precision, rows, ld).  The engine's own GEMM buffers serve as operands
// before its first step.  The split-BF16 GEMM is not tuned (default launch).
// LYAP_GEMM_TUNE_LOG=1 prints the candidate table to stderr.
namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, long long, long long>, GemmTune> g_tune;
GemmTune g_last_tune;
}  // namespace

static GemmTune tune_cauchy(lyap_engine_s* E, GemmType type) {
  const long long ld = E->sd->ld, rows = E->rows_pad;
  const GemmTune dflt{type == GemmType::F64 ? 16 : 32, (long long)kSkGridMults[0] * kSkGridUnit, 1};
  if (type == GemmType::BF16X3) return dflt;
  // LYAP_GEMM_CONFIG="bk,grid_mult,xcd_off" fixes the configuration (tests,
  // diagnostics): bk one of the precision's K-tile depths, grid_mult 2 or 4
  // (workgroups per CU of a 256-CU device)
  if (const char* env = std::getenv("LYAP_GEMM_CONFIG")) {
    int bk = 0, mult = 0, xoff = 0;
    LYAP_REQUIRE(std::sscanf(env, "%d,%d,%d", &bk, &mult, &xoff) == 3, LYAP_E_INVAL,
                 "LYAP_GEMM_CONFIG must be bk,grid_mult,xcd_off");
    const bool ok_bk = type == GemmType::F64 ? (bk == 8 || bk == 16) : (bk == 16 || bk == 32);
    const bool ok_mult = mult == kSkGridMults[0] || mult == kSkGridMults[1];
    LYAP_REQUIRE(ok_bk && ok_mult && (xoff == 0 || xoff == 1), LYAP_E_INVAL,
                 "LYAP_GEMM_CONFIG out of the candidate set");
    return GemmTune{bk, (long long)mult * kSkGridUnit, xoff};
  }
  const auto key = std::make_tuple((int)type, rows, ld);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return it->second;
  }
  hipStream_t st = E->stream;
  const int bks[2] = {type == GemmType::F64 ? 8 : 16, type == GemmType::F64 ? 16 : 32};
  std::vector<GemmTune> cand;
  cand.push_back(dflt);  // the default launch comes first
  for (int bk : bks)
    for (int mult : kSkGridMults)
      for (int x : {0, 1}) {
        const GemmTune c{bk, (long long)mult * kSkGridUnit, x};
        if (!(c.bk == dflt.bk && c.grid_min == dflt.grid_min && c.xcd_off == dflt.xcd_off))
          cand.push_back(c);
      }
  const bool log = std::getenv("LYAP_GEMM_TUNE_LOG") != nullptr;
  const long long full = rows;
  const long long regimes[3] = {full, std::max<long long>(kGemmBM, (full / 8) / kGemmBM * kGemmBM),
                                std::min<long long>(full, 32)};
  const double weight[3] = {0.15, 0.15, 0.7};
  DevBuf mdev(sizeof(int));
  hipEvent_t e0, e1;
  LYAP_HIP(hipEventCreate(&e0));
  LYAP_HIP(hipEventCreate(&e1));
  GemmTune best{};
  double best_t = 1e300, default_t = 0;
  try {
    for (size_t ci = 0; ci < cand.size(); ++ci) {
      const GemmTune& c = cand[ci];
      GemmArgs g{};
      g.type = type;
      g.A = type == GemmType::F64 ? E->X.p : E->Xlo.p;
      g.B = type == GemmType::F64 ? E->sd->Mc.p : E->sd->Mc32.p;
      g.C = type == GemmType::F64 ? E->H.p : E->Hlo.p;
      g.M = rows;
      g.N = ld;
      g.K = ld;
      g.lda = g.ldb = g.ldc = ld;
      g.Nstore = ld;
      g.M_dev = mdev.as<int>();
      g.m_scale = 1;
      g.Cpart = type == GemmType::F64 ? E->Hp.p : E->Hplo.p;
      g.Cpart_rows = cauchy_part_rows(rows, ld, type);
      g.bk = c.bk;
      g.grid_min = c.grid_min;
      g.xcd_off = c.xcd_off;
      g.tuning = 1;
      g.streamk = 1;
      double tot = 0, per[3];
      for (int q = 0; q < 3; ++q) {
        const int m = (int)regimes[q];
        LYAP_HIP(hipMemcpy(mdev.p, &m, sizeof(int), hipMemcpyHostToDevice));
        gemm_launch(g, st);
        float t[5];
        for (int rep = 0; rep < 5; ++rep) {
          LYAP_HIP(hipEventRecord(e0, st));
          gemm_launch(g, st);
          gemm_launch(g, st);
          LYAP_HIP(hipEventRecord(e1, st));
          LYAP_HIP(hipEventSynchronize(e1));
          LYAP_HIP(hipEventElapsedTime(&t[rep], e0, e1));
        }
        std::sort(t, t + 5);
        per[q] = t[2] / 2;
        tot += weight[q] * per[q];
      }
      if (log)
        std::fprintf(stderr, "gemm tune rows=%lld ld=%lld bk=%d grid_min=%lld xcd_off=%d: "
                     "full %.1f us, 1/8 %.1f us, tail %.1f us, weighted %.1f us\n",
                     rows, ld, c.bk, c.grid_min, c.xcd_off, 1e3 * per[0], 1e3 * per[1],
                     1e3 * per[2], 1e3 * tot);
      if (ci == 0) {
        default_t = tot;
        best_t = tot;
        best = c;
      } else if (tot < best_t && tot < 0.97 * default_t) {
        best_t = tot;
        best = c;
      }
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[key] = best;
  return best;
}

// ws: optional caller workspace of at least engine_sizes(...).total bytes; the
// engine's buffers are then carved from it (no device allocation here).
static lyap_engine_s* engine_create_impl(lyap_seed_s* sd, long long S, const lyap_solve_opts* in,
                                         hipStream_t st, long long Q, double* sol,
                                         long long sol_cap, bool use_graph, void* ws = nullptr) {
  LYAP_REQUIRE(sd != nullptr, LYAP_E_INVAL, "seed is NULL");
  LYAP_REQUIRE(S >= 1 && S <= 8192, LYAP_E_INVAL, "slots out of [1, 8192]");
  lyap_solve_opts o;
  fill_defaults(o, in);
  validate_opts(o);
  auto* E = new lyap_engine_s();
  std::unique_ptr<lyap_engine_s> guard(E);
  E->sd = sd;
  E->S = (int)S;
  E->m = o.restart;
  E->opts = o;
  LYAP_HIP(hipStreamCreateWithFlags(&E->stream, hipStreamNonBlocking));
  {
    // order the engine after the caller's stream
    hipEvent_t ev;
    LYAP_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    LYAP_HIP(hipEventRecord(ev, st));
    LYAP_HIP(hipStreamWaitEvent(E->stream, ev, 0));
    LYAP_HIP(hipEventDestroy(ev));
  }
  st = E->stream;
  E->mixed = o.prec != LYAP_PREC_FP64;
  LYAP_REQUIRE(!(E->mixed && sd->basis == LYAP_BASIS_SCHUR), LYAP_E_UNSUPPORTED,
               "the Schur-basis seed solve runs in FP64 only");
  E->low = o.prec == LYAP_PREC_BF16_IR ? GemmType::BF16X3 : GemmType::F32;
  E->Q = (int)Q;
  const long long r = sd->r, ld = sd->ld, N = slot_stride(r, ld), m = o.restart;
  EngineSizes z = engine_sizes(sd, S, o, Q);
  // the consumers of the Cauchy GEMM's stream-K partials index its
  // (tile, K-tile) iterations in 32 bits
  LYAP_REQUIRE((z.rows_pad / kGemmBM + 1) * (ld / kGemmBN) * (ld / 8) < (1LL << 31), LYAP_E_INVAL,
               "Cauchy GEMM too large for 32-bit stream-K indices");
  E->rows_pad = z.rows_pad;
  size_t carve = 0;
  engine_layout(sd, S, o, Q, E, [&](DevBuf* b, size_t bytes) {
    bytes = std::max<size_t>(bytes, 16);
    if (ws) {
      b->view(static_cast<char*>(ws) + carve, bytes);
      carve += (bytes + 255) / 256 * 256;
    } else {
      b->alloc(bytes);
    }
    LYAP_HIP(hipMemsetAsync(b->p, 0, b->bytes, st));
  });
  E->sol = sol;
  E->sol_cap = sol_cap;
  E->ws = ws;
  E->res_host.resize(Q);
  E->got.assign(Q, 0);

  EngineArgs& A = E->args;
  A.Uh = sd->Uh.as<double>();
  A.Vh = sd->Vh.as<double>();
  A.K1 = sd->K1.as<double>();
  A.c0 = sd->c0.as<double>();
  A.gam = sd->gam.as<double>();
  A.t0 = sd->t0;
  A.eps_seed = sd->eps_seed;
  A.n = (int)sd->n;
  A.h = (int)sd->h;
  A.ld = (int)ld;
  A.r = (int)r;
  A.NV = (int)N;
  A.S = (int)S;
  A.m = (int)m;
  A.max_iter = o.max_iter;
  A.max_refine = o.max_refine;
  A.use_precond = (o.use_precond && r <= kPrecRank && sd->basis != LYAP_BASIS_SCHUR) ? 1 : 0;
  // use_precond 1: all of eq:prec the seed holds; 2: its block-diagonal part only
  const bool tsvd = sd->pbar > 0 && o.use_precond == 1 && r <= kPrecRank;
  A.pbar = tsvd ? (int)sd->pbar : 0;
  A.Ks = (int)(r * ld);
  A.TsM = sd->TsM.as<double>();
  A.TsN = sd->TsN.as<double>();
  A.Cpinv = E->Cpinv.as<double>();
  A.Yc = E->X.as<double>();
  A.Qc = E->H.as<double>();
  A.Tbuf = E->Tbuf.as<double>();
  A.Tpart = E->Tpart.as<double>();
  A.Sc = E->Sc.as<double>();
  A.mixed = E->mixed ? 1 : 0;
  A.tol = o.tol;
  A.inner_tol = o.inner_tol;
  A.si = E->si.as<int>();
  A.sdv = E->sdv.as<double>();
  A.d = E->d.as<double>();
  A.R = E->R.as<double>();
  A.g = E->g.as<double>();
  A.cs = E->cs.as<double>();
  A.sn = E->sn.as<double>();
  A.V = E->V.as<double>();
  A.x = E->x.as<double>();
  A.z = E->z.as<double>();
  A.w = E->w.as<double>();
  A.Pinv = E->Pinv.as<double>();
  A.nchunk = (int)(N / (2 * orth_threads(N)));
  A.orth1 = E->orth1.as<double>();
  A.orth1b = E->orth1b.as<double>();
  A.ycoefs = E->ycoefs.as<double>();
  A.orthA = E->orthA.as<double>();
  A.coefB = E->coefB.as<double>();
  A.Hu = E->Hu.as<double>();
  if (const char* env = std::getenv("LYAP_EPI_GRID")) E->egrid = std::max(1, std::atoi(env));
  if (const char* env = std::getenv("LYAP_ORTH_GRID")) E->og_cap = std::max(1, std::atoi(env));
  // LYAP_ORTH=cgs2 selects classical CGS2 in three passes (measurements)
  A.dcgs = orth_dcgs() ? 1 : 0;
  A.vf32 = basis_f32(o) ? 1 : 0;
  A.Vf = E->Vf.as<float>();
  A.orth2 = E->orth2.as<double>();
  A.lists = E->lists.as<int>();
  A.qd = E->qd.as<double>();
  A.qtag = E->qtag.as<long long>();
  A.qctl = E->qctl.as<int>();
  A.res = E->res.as<DevResult>();
  A.Q = (int)Q;
  A.sol = sol;
  A.sol_cap = sol_cap;
  A.kmax = o.recycle_k;
  A.Ur = E->Ur.as<double>();
  A.Cr = E->Cr.as<double>();
  A.Bk = E->Bk.as<double>();
  A.Hr = E->Hr.as<double>();
  A.Fs = E->Fs.as<double>();
  LYAP_HIP(hipStreamSynchronize(st));
  if (sd->basis != LYAP_BASIS_SCHUR) {
    E->t64 = tune_cauchy(E, GemmType::F64);
    if (E->mixed) E->tlo = tune_cauchy(E, E->low);
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_last_tune = E->t64;
  }

  if (use_graph) {
    LYAP_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
      launch_step(E, st);
    } catch (...) {
      hipGraph_t tmp;
      (void)hipStreamEndCapture(st, &tmp);
      throw;
    }
    LYAP_HIP(hipStreamEndCapture(st, &E->graph));
    LYAP_HIP(hipGraphInstantiate(&E->gexec, E->graph, nullptr, nullptr, 0));
    E->owns_graph = true;
  }
  guard.release();
  return E;
}

static void engine_destroy_impl(lyap_engine_s* E) {
  if (!E) return;
  (void)hipStreamSynchronize(E->stream);
  if (E->gexec) (void)hipGraphExecDestroy(E->gexec);
  if (E->graph) (void)hipGraphDestroy(E->graph);
  for (int q = 0; q < 3; ++q) {
    if (E->psegx[q]) (void)hipGraphExecDestroy(E->psegx[q]);
    if (E->pseg[q]) (void)hipGraphDestroy(E->pseg[q]);
  }
  for (auto& e : E->pev) (void)hipEventDestroy(e);
  if (E->stream) (void)hipStreamDestroy(E->stream);
  delete E;
}

// Back to the state of a new engine (free slots, empty queue, no recycle
// space), ordered after the caller's stream; buffers and graphs are kept.
static void engine_reset(lyap_engine_s* E, hipStream_t user) {
  hipStream_t st = E->stream;
  hipEvent_t ev;
  LYAP_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  LYAP_HIP(hipEventRecord(ev, user));
  LYAP_HIP(hipStreamWaitEvent(st, ev, 0));
  LYAP_HIP(hipEventDestroy(ev));
  LYAP_HIP(hipMemsetAsync(E->si.p, 0, E->si.bytes, st));
  LYAP_HIP(hipMemsetAsync(E->lists.p, 0, E->lists.bytes, st));  // no slot listed
  LYAP_HIP(hipMemsetAsync(E->qctl.p, 0, E->qctl.bytes, st));
  LYAP_HIP(hipMemsetAsync(E->res.p, 0, E->res.bytes, st));
  E->submitted = E->harvested = E->next_tag = 0;
  E->got.assign(E->Q, 0);
  E->done_pos.clear();
}

// host -> device queue append (positions submitted .. submitted+count)
static void engine_submit_impl(lyap_engine_s* E, long long count, const double* d_host,
                               const long long* tags) {
  LYAP_REQUIRE(count >= 0, LYAP_E_INVAL, "count < 0");
  if (count == 0) return;
  LYAP_REQUIRE(d_host != nullptr, LYAP_E_INVAL, "d is NULL");
  const long long inflight = E->submitted - E->harvested;
  LYAP_REQUIRE(inflight + count <= E->Q, LYAP_E_INVAL, "engine queue capacity exceeded");
  const int r = (int)E->sd->r;
  hipStream_t st = E->stream;
  // copy in at most two contiguous pieces of the ring
  long long done = 0;
  std::vector<long long> tg(count);
  for (long long i = 0; i < count; ++i) tg[i] = tags ? tags[i] : E->next_tag + i;
  while (done < count) {
    const long long pos = (E->submitted + done) % E->Q;
    const long long piece = std::min(count - done, (long long)E->Q - pos);
    LYAP_HIP(hipMemcpyAsync(E->qd.as<double>() + pos * r, d_host + done * r,
                            piece * r * sizeof(double), hipMemcpyHostToDevice, st));
    LYAP_HIP(hipMemcpyAsync(E->qtag.as<long long>() + pos, tg.data() + done,
                            piece * sizeof(long long), hipMemcpyHostToDevice, st));
    // clear result records of the new positions
    LYAP_HIP(hipMemsetAsync(E->res.as<DevResult>() + pos, 0, piece * sizeof(DevResult), st));
    done += piece;
  }
  E->submitted += count;
  if (!tags) E->next_tag += count;
  const int tail = (int)(E->submitted);
  LYAP_HIP(hipMemcpyAsync(E->qctl.as<int>() + 1, &tail, sizeof(int), hipMemcpyHostToDevice, st));
  LYAP_HIP(hipStreamSynchronize(st));  // tail lives on the host stack
}

static long long engine_done_count(lyap_engine_s* E) {
  int c = 0;
  LYAP_HIP(hipMemcpyAsync(&c, E->qctl.as<int>() + 2, sizeof(int), hipMemcpyDeviceToHost, E->stream));
  LYAP_HIP(hipStreamSynchronize(E->stream));
  return c;
}

static long long engine_run_impl(lyap_engine_s* E, long long max_steps, int poll_every) {
  if (poll_every < 1) poll_every = 8;
  long long steps = 0;
  while (steps < max_steps) {
    const long long busy = E->submitted - engine_done_count(E);
    if (busy <= 0) return 0;
    const long long k = std::min<long long>(poll_every, max_steps - steps);
    const int level = profiling();
    if (level) {
      profiled_steps(E, k, level);
    } else {
      for (long long i = 0; i < k; ++i) {
        if (E->gexec) LYAP_HIP(hipGraphLaunch(E->gexec, E->stream));
        else launch_step(E, E->stream);
      }
    }
    steps += k;
  }
  return E->submitted - engine_done_count(E);
}

static long long engine_harvest_impl(lyap_engine_s* E, long long max_out, long long* tags_out,
                                     lyap_result* res_out) {
  // copy the records of all in-flight positions (ring order)
  const long long lo = E->harvested, hi = E->submitted;
  if (hi <= lo || max_out <= 0) return 0;
  for (long long p = lo; p < hi;) {
    const long long pos = p % E->Q;
    const long long piece = std::min(hi - p, (long long)E->Q - pos);
    LYAP_HIP(hipMemcpyAsync(E->res_host.data() + pos, E->res.as<DevResult>() + pos,
                            piece * sizeof(DevResult), hipMemcpyDeviceToHost, E->stream));
    p += piece;
  }
  LYAP_HIP(hipStreamSynchronize(E->stream));
  long long n = 0;
  for (long long p = lo; p < hi && n < max_out; ++p) {
    const long long pos = p % E->Q;
    const DevResult& o = E->res_host[pos];
    if (!o.valid || E->got[pos]) continue;
    E->got[pos] = 1;
    if (tags_out) tags_out[n] = o.tag;
    if (res_out) {
      res_out[n].status = o.status;
      res_out[n].iters = o.iters;
      res_out[n].cycles = o.cycles;
      res_out[n].refinements = o.refines;
      res_out[n].rel_residual = o.relres;
      res_out[n].err_est = o.err_est;
      res_out[n].trace = o.trace;
    }
    ++n;
  }
  // advance the harvested watermark over contiguous harvested positions
  while (E->harvested < E->submitted && E->got[E->harvested % E->Q]) {
    E->got[E->harvested % E->Q] = 0;
    ++E->harvested;
  }
  return n;
}

}  // namespace lyap


static long long default_slots(const lyap_seed_s* sd, long long P) {
  if (sd->basis == LYAP_BASIS_SCHUR && !sd->Kd.p) {
    // one n x n solution per slot: bound the buffer by 4 GiB
    const long long per = sd->ld * sd->ld * 8;
    const long long S = std::max<long long>(1, std::min<long long>(512, (4LL << 30) / per));
    return std::max<long long>(1, std::min(S, P));
  }
  // enough rows for the Cauchy GEMM to fill the GPU, bounded by P
  const long long r = sd->r;
  long long S = std::max<long long>(64, 8192 / (r * r));
  S = std::min<long long>(S, 2048);
  return std::max<long long>(1, std::min(S, P));
}

namespace lyap {

// Run P parameters (device d, tags 0..P-1) through an engine whose queue and
// solution store hold at least P, then write the physical solutions
// Y = rho(Yhat) Tout to Y_dev (P x r x n) and the results to res_host.
// The engine must have been reset (or freshly created) on the caller's stream.
void engine_batch_run(lyap_engine_s* E, long long P, const double* d_dev, double* Y_dev,
                      lyap_result* res_host) {
  lyap_seed_s* sd = E->sd;
  LYAP_REQUIRE(P >= 1 && P <= E->Q && P <= E->sol_cap, LYAP_E_INVAL, "batch exceeds the engine");
  const long long r = sd->r, ld = sd->ld, n = sd->n, S = E->S;
  const lyap_solve_opts o = E->opts;
  double* sol = E->sol;
  hipStream_t st = E->stream;
  // queue: d from device, tags 0..P-1
  LYAP_HIP(hipMemcpyAsync(E->qd.p, d_dev, P * r * sizeof(double), hipMemcpyDeviceToDevice, st));
  std::vector<long long> tags(P);
  for (long long i = 0; i < P; ++i) tags[i] = i;
  LYAP_HIP(hipMemcpyAsync(E->qtag.p, tags.data(), P * sizeof(long long), hipMemcpyHostToDevice, st));
  const int tail = (int)P;
  LYAP_HIP(hipMemcpyAsync(E->qctl.as<int>() + 1, &tail, sizeof(int), hipMemcpyHostToDevice, st));
  LYAP_HIP(hipStreamSynchronize(st));
  E->submitted = P;
  const long long max_steps = (long long)o.max_iter * ((P + S - 1) / S + 1) + 16;
  engine_run_impl(E, max_steps, 8);
  std::vector<long long> tg(P);
  std::vector<lyap_result> rr(P);
  const long long got = engine_harvest_impl(E, P, tg.data(), rr.data());
  for (long long i = 0; i < P; ++i) res_host[i] = lyap_result{LYAP_E_NOCONV, 0, 0, 0, NAN, NAN, NAN};
  for (long long i = 0; i < got; ++i)
    if (tg[i] >= 0 && tg[i] < P) res_host[tg[i]] = rr[i];
  // physical Y = rho(Yhat) Tout  (transform-out GEMM, n columns stored)
  GemmArgs g{};
  g.type = GemmType::F64;
  g.A = sol;
  g.B = sd->Tout.p;
  g.C = Y_dev;
  g.M = P * r;
  g.N = ld;
  g.K = ld;
  g.lda = ld;
  g.ldb = ld;
  g.ldc = n;
  g.Nstore = n;
  g.M_dev = nullptr;
  g.m_scale = 1;
  gemm_launch(g, st);
  LYAP_HIP(hipStreamSynchronize(st));
}

// Engines owned by other parts of the library (one batch size cap, one store).
lyap_engine_s* engine_batch_create(lyap_seed_s* sd, long long P_cap, const lyap_solve_opts* opts,
                                   hipStream_t st, double* sol) {
  lyap_solve_opts o;
  fill_defaults(o, opts);
  validate_opts(o);
  return engine_create_impl(sd, default_slots(sd, P_cap), &o, st, P_cap, sol, P_cap, true);
}
void engine_batch_reset(lyap_engine_s* E, hipStream_t st) { engine_reset(E, st); }
void engine_batch_destroy(lyap_engine_s* E) { engine_destroy_impl(E); }
bool engine_batch_fits(const lyap_engine_s* E, long long P, const lyap_solve_opts* opts) {
  lyap_solve_opts o;
  fill_defaults(o, opts);
  return P <= E->Q && P <= E->sol_cap && std::memcmp(&o, &E->opts, sizeof(o)) == 0;
}

}  // namespace lyap

extern "C" {

size_t engine_device_bytes(lyap_seed sd, int64_t slots, const lyap_solve_opts* opts) {
  if (!sd || slots < 1) return 0;
  try {
    lyap_solve_opts o;
    fill_defaults(o, opts);
    return engine_sizes(sd, slots, o, std::max<int64_t>(4 * slots, 1024)).total;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return 0;
  }
}

lyap_status engine_create(lyap_seed sd, int64_t slots, const lyap_solve_opts* opts,
                          void* hip_stream, lyap_engine* out) {
  if (!out) return LYAP_E_INVAL;
  *out = nullptr;
  LYAP_TRY(*out = engine_create_impl(sd, slots, opts, (hipStream_t)hip_stream,
                                     std::max<int64_t>(4 * slots, 1024), nullptr, 0, true));
  return LYAP_OK;
}

lyap_status engine_destroy(lyap_engine E) {
  if (!E) return LYAP_E_INVAL;
  LYAP_TRY(engine_destroy_impl(E));
  return LYAP_OK;
}

lyap_status engine_submit(lyap_engine E, int64_t count, const double* d_host, const int64_t* tags) {
  if (!E) return LYAP_E_INVAL;
  LYAP_TRY(engine_submit_impl(E, count, d_host, reinterpret_cast<const long long*>(tags)));
  return LYAP_OK;
}

lyap_status engine_run(lyap_engine E, int64_t max_steps, int32_t poll_every, int64_t* busy) {
  if (!E) return LYAP_E_INVAL;
  LYAP_TRY({
    const long long b = engine_run_impl(E, max_steps, poll_every);
    if (busy) *busy = b;
  });
  return LYAP_OK;
}

lyap_status engine_launch(lyap_engine E, int64_t steps) {
  if (!E || steps < 0) return LYAP_E_INVAL;
  LYAP_TRY({
    for (int64_t i = 0; i < steps; ++i) {
      if (E->gexec) LYAP_HIP(hipGraphLaunch(E->gexec, E->stream));
      else launch_step(E, E->stream);
    }
  });
  return LYAP_OK;
}

lyap_status engine_status(lyap_engine E, int64_t* submitted, int64_t* done) {
  if (!E) return LYAP_E_INVAL;
  LYAP_TRY({
    const long long d = engine_done_count(E);
    if (submitted) *submitted = E->submitted;
    if (done) *done = d;
  });
  return LYAP_OK;
}

lyap_status engine_harvest(lyap_engine E, int64_t max_out, int64_t* tags_out, lyap_result* res_out,
                           int64_t* n_out) {
  if (!E) return LYAP_E_INVAL;
  LYAP_TRY({
    const long long n =
        engine_harvest_impl(E, max_out, reinterpret_cast<long long*>(tags_out), res_out);
    if (n_out) *n_out = n;
  });
  return LYAP_OK;
}

void lyap_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_level = on < 0 ? 0 : (on > 2 ? 2 : on);
  g_prof = lyap_profile{};
}

lyap_status lyap_profile_read(lyap_profile* out) {
  if (!out) return LYAP_E_INVAL;
  GemmTune t;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    t = g_last_tune;
  }
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof.tuned_bk = t.bk;
  g_prof.tuned_grid_min = t.grid_min;
  g_prof.tuned_xcd_off = t.xcd_off;
  *out = g_prof;
  return LYAP_OK;
}

size_t smw_workspace_bytes(lyap_seed sd, int64_t P, const lyap_solve_opts* opts) {
  if (!sd || P < 1) return 0;
  try {
    lyap_solve_opts o;
    fill_defaults(o, opts);
    const long long S = default_slots(sd, P);
    const size_t sol = (size_t)P * sd->r * sd->ld * sizeof(double);
    return engine_sizes(sd, S, o, P).total + sol;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return 0;
  }
}

lyap_status smw_solve_batch(lyap_seed sd, int64_t P, const double* d_dev,
                            const lyap_solve_opts* opts, double* Y_dev, lyap_result* res_host,
                            void* workspace_dev, size_t workspace_bytes, void* hip_stream) {
  if (!sd || P < 1 || !d_dev || !Y_dev || !res_host) return LYAP_E_INVAL;
  LYAP_TRY({
    lyap_solve_opts o;
    fill_defaults(o, opts);
    validate_opts(o);
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t need = smw_workspace_bytes(sd, P, opts);
    LYAP_REQUIRE(need > 0, LYAP_E_INVAL, lyap_last_error());
    LYAP_REQUIRE(workspace_dev == nullptr || workspace_bytes >= need, LYAP_E_INVAL,
                 "workspace too small");
    LYAP_REQUIRE(workspace_dev == nullptr || ((uintptr_t)workspace_dev & 255) == 0,
                 LYAP_E_INVAL, "workspace must be 256-byte aligned");
    const long long r = sd->r, ld = sd->ld;
    const long long S = default_slots(sd, P);
    const size_t eng_bytes = engine_sizes(sd, S, o, P).total;
    // The engine (buffers, captured step graphs) is kept on the seed for the next
    // call with the same slots, length, options and memory.  With a workspace,
    // every engine buffer and the solution store are carved from it (the next
    // call with the same workspace allocates nothing); without one, the seed
    // allocates and owns them.  A call that finds the cache in use by another
    // thread builds a private engine.
    std::unique_lock<std::mutex> lk(sd->cache_mu, std::try_to_lock);
    DevBuf own;
    double* sol;
    void* ews = nullptr;
    if (workspace_dev) {
      ews = workspace_dev;
      sol = reinterpret_cast<double*>(static_cast<char*>(workspace_dev) + eng_bytes);
    } else if (lk.owns_lock()) {
      const size_t b = (size_t)P * r * ld * sizeof(double);
      if (sd->sol_buf.bytes < b) {
        if (sd->eng_cache) {  // the cached engine refers to the old store
          engine_destroy_impl(reinterpret_cast<lyap_engine_s*>(sd->eng_cache));
          sd->eng_cache = nullptr;
        }
        sd->sol_buf.alloc(b);
      }
      sol = sd->sol_buf.as<double>();
    } else {
      own.alloc((size_t)P * r * ld * sizeof(double));
      sol = own.as<double>();
    }
    std::unique_ptr<lyap_engine_s, void (*)(lyap_engine_s*)> eg(nullptr, engine_destroy_impl);
    lyap_engine_s* E = nullptr;
    if (lk.owns_lock()) {
      auto* C = reinterpret_cast<lyap_engine_s*>(sd->eng_cache);
      if (C && C->S == S && C->Q == P && C->sol == sol && C->sol_cap == P && C->ws == ews &&
          std::memcmp(&C->opts, &o, sizeof(o)) == 0) {
        E = C;
        engine_reset(E, st);
      } else {
        if (C) engine_destroy_impl(C);
        sd->eng_cache = nullptr;
        E = engine_create_impl(sd, S, &o, st, P, sol, P, true, ews);
        sd->eng_cache = E;
        sd->eng_cache_free = [](void* q) { engine_destroy_impl(reinterpret_cast<lyap_engine_s*>(q)); };
        sd->eng_cache_bytes = [](const void* q) {
          const auto* e = reinterpret_cast<const lyap_engine_s*>(q);
          return e->ws ? size_t(0) : engine_sizes(e->sd, e->S, e->opts, e->Q).total;
        };
      }
    } else {
      E = engine_create_impl(sd, S, &o, st, P, sol, P, true, ews);
      eg.reset(E);
    }
    engine_batch_run(E, P, d_dev, Y_dev, res_host);
  });
  return LYAP_OK;
}

}  // extern "C"
