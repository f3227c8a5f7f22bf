// MFMA GEMM kernels for gfx950 (CDNA4).
//
// One GEMM shape serves the whole library: C[M x N] = A[M x K] * B[K x N],
// row-major, with K and N padded to the tile so the inner loop has no bounds
// checks.  It carries both the basis transforms (A = batched r x n blocks, B =
// the real eigenbasis or its inverse) and the Cauchy contraction of the seed
// Lyapunov solve (A = Hadamard products of low-rank rows, B = the real form of
// the Cauchy matrix 1/(lambda_i + lambda_j)).
//
// Tiling: 128 x 128 workgroup tile, 4 waves of 64 x 64, 16 x 16 MFMA blocks.
// Operands are staged through LDS with one barrier per K-tile (double buffer);
// the next K-tile is fetched into registers while the current one is
// multiplied.  Workgroups are mapped to tiles so that consecutive tiles of one
// B column panel land on the same XCD (blocks are dispatched round-robin over
// the 8 XCDs), which keeps the shared B panel in that XCD's L2.
//
// The engine's Cauchy GEMMs run as stream-K launches (sk_plan): a fixed grid
// of two workgroups per CU shares the (tile, K-tile) iterations of the active
// rows evenly, and the consumer adds the partial tiles.
#include <algorithm>

#include "common.h"

namespace lyap {

namespace {

constexpr int BM = 128;
constexpr int BN = 128;
constexpr int NTHREADS = 256;

typedef double double4_ __attribute__((ext_vector_type(4)));
typedef float float4_ __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_ __attribute__((ext_vector_type(8)));

__device__ inline double4_ mfma(double a, double b, double4_ c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline float4_ mfma(float a, float b, float4_ c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <class T> struct Acc;
template <> struct Acc<double> { typedef double4_ type; };
template <> struct Acc<float> { typedef float4_ type; };

// Tile index -> (m-tile, n-tile), with XCD-aware grouping unless xcd == 0.
__device__ inline void tile_of(int bid, int mtiles, int ntiles, int& mt, int& nt, int xcd = 1) {
  const int T = mtiles * ntiles;
  int t = bid;
  const int full = (T / 8) * 8;
  if (xcd && bid < full) {
    const int per = full / 8;
    t = (bid % 8) * per + bid / 8;
  }
  nt = t / mtiles;
  mt = t % mtiles;
}

// ---------------------------------------------------------------------------
// FP64 / FP32: v_mfma_{f64,f32}_16x16x4.  Lane layout (16 x 16 x 4):
//   A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k,
//   D[i][j]: f32 in lane j + 16 (i / 4), element i % 4;
//            f64 in lane j + 16 (i % 4), element i / 4 (measured on gfx950).
// LDS holds A transposed (k-major) so a fragment read is 16 consecutive rows.
// ---------------------------------------------------------------------------
// One output tile of BMV rows (128, or 64 / 32 for few active rows) at
// (row0, col0) over the K-tiles [k0, k1): C rows below Meff and columns below
// Nstore are stored.  Waves 2 x 2, each BMV / 2 rows x 64 columns.  Leaves
// LDS free for the next call (the last K-tile ends with a barrier).
template <class T, int BK, int PAD, int BMV = BM>
__device__ inline void mac_tile(const T* __restrict__ A, const T* __restrict__ B, T* __restrict__ C,
                                int M, int Meff, int row0, int col0, int k0, int k1, long lda,
                                long ldb, long ldc, int Nstore, T (&As)[2][BK][BM + PAD],
                                T (&Bs)[2][BK][BN + PAD]) {
  typedef typename Acc<T>::type acc_t;
  constexpr int IM = BMV / 32;  // 16-row blocks per wave
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave >> 1) * (BMV / 2);
  const int wn0 = (wave & 1) * 64;

  // global -> register mapping
  constexpr int A_PER = BMV * BK / NTHREADS;     // elements per thread
  constexpr int A_TPR = BK / A_PER;              // threads per row
  const int a_row = tid / A_TPR;
  const int a_k = (tid % A_TPR) * A_PER;
  int a_grow = row0 + a_row;
  if (a_grow > M - 1) a_grow = M - 1;
  const T* a_src = A + (long)a_grow * lda + a_k;

  constexpr int B_PER = BK * BN / NTHREADS;
  constexpr int B_TPR = BN / B_PER;
  const int b_k = tid / B_TPR;
  const int b_n = (tid % B_TPR) * B_PER;
  const T* b_src = B + (long)b_k * ldb + col0 + b_n;

  T ra[A_PER], rb[B_PER];

  auto gload = [&](int kt) {
    const T* pa = a_src + (long)kt * BK;
#pragma unroll
    for (int i = 0; i < A_PER; ++i) ra[i] = pa[i];
    const T* pb = b_src + (long)kt * BK * ldb;
#pragma unroll
    for (int i = 0; i < B_PER; ++i) rb[i] = pb[i];
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < A_PER; ++i) As[buf][a_k + i][a_row] = ra[i];
#pragma unroll
    for (int i = 0; i < B_PER; ++i) Bs[buf][b_k][b_n + i] = rb[i];
  };

  acc_t acc[IM][4];
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  gload(k0);
  sstore(0);
  __syncthreads();
  const int lr = lane & 15;
  const int lk = lane >> 4;
  for (int kt = k0; kt < k1; ++kt) {
    const int cur = (kt - k0) & 1;
    if (kt + 1 < k1) gload(kt + 1);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T af[IM], bfr[4];
#pragma unroll
      for (int i = 0; i < IM; ++i) af[i] = As[cur][kk + lk][wm0 + 16 * i + lr];
#pragma unroll
      for (int j = 0; j < 4; ++j) bfr[j] = Bs[cur][kk + lk][wn0 + 16 * j + lr];
#pragma unroll
      for (int i = 0; i < IM; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma(af[i], bfr[j], acc[i][j]);
    }
    if (kt + 1 < k1) sstore(cur ^ 1);
    __syncthreads();
  }

  // output rows of element v: f64 16x16x4 -> lane/16 + 4 v ; f32 16x16x4 -> 4 (lane/16) + v
  constexpr bool kF64 = sizeof(T) == 8;
#pragma unroll
  for (int i = 0; i < IM; ++i) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = row0 + wm0 + 16 * i + (kF64 ? lk + 4 * v : 4 * lk + v);
      if (row >= Meff) continue;
      T* crow = C + (long)row * ldc;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = col0 + wn0 + 16 * j + lr;
        if (col < Nstore) crow[col] = acc[i][j][v];
      }
    }
  }
}

// TUNE only separates the autotuner's timing launches from production
// launches in kernel traces (same code, distinct symbol).
template <class T, int BK, bool TUNE = false>
__global__ void __launch_bounds__(NTHREADS, 2)  // two workgroups per CU (the stream-K grid)
gemm_kernel(const T* __restrict__ A, const T* __restrict__ B, T* __restrict__ C,
            int M, int N, int K, long lda, long ldb, long ldc, int Nstore,
            const int* __restrict__ M_dev, int m_scale, T* __restrict__ Cpart, int xcd,
            int streamk) {
  constexpr int PAD = 4;
  __shared__ T As[2][BK][BM + PAD];
  __shared__ T Bs[2][BK][BN + PAD];

  const int mtiles = (M + BM - 1) / BM;
  const int ntiles = N / BN;
  int Meff = M;
  if (M_dev) {
    const int md = M_dev[0] * m_scale;
    Meff = md < M ? md : M;
  }
  const int nk_all = K / BK;
  if (streamk) {
    const SkPlan p = sk_plan(Meff, ntiles, (int)gridDim.x, nk_all);
    const int v = sk_range_of(blockIdx.x, gridDim.x, xcd);
    long long it, end;
    sk_range(p, v, it, end);
    const long segstride = (long)p.mta * p.bm * ldc;
    while (it < end) {
      int t, k0, k1, s0, ns;
      sk_piece(p, it, end, t, k0, k1);
      sk_segments(p, t, s0, ns);
      T* dst = Cpart + (long)(v - s0) * segstride;
      const int row0 = (t % p.mta) * p.bm, col0 = (t / p.mta) * BN;
      const int hb = sk_tile_height(p, t % p.mta, Meff);
      if (hb == 32)
        mac_tile<T, BK, PAD, 32>(A, B, dst, M, Meff, row0, col0, k0, k1, lda, ldb, ldc, Nstore, As, Bs);
      else if (hb == 64)
        mac_tile<T, BK, PAD, 64>(A, B, dst, M, Meff, row0, col0, k0, k1, lda, ldb, ldc, Nstore, As, Bs);
      else
        mac_tile<T, BK, PAD>(A, B, dst, M, Meff, row0, col0, k0, k1, lda, ldb, ldc, Nstore, As, Bs);
      it += k1 - k0;
    }
    return;
  }
  int mt, nt, ks = 0, KS = 1;
  if (Cpart) {
    const int mta = (Meff + BM - 1) / BM;
    KS = splitk_of(mta, ntiles, (int)gridDim.x, nk_all);
    if (KS > 1) {
      const int tiles = mta * ntiles;
      if ((int)blockIdx.x >= tiles * KS) return;
      const int t = blockIdx.x % tiles;
      ks = blockIdx.x / tiles;
      nt = t / mta;
      mt = t % mta;
    } else {
      tile_of(blockIdx.x, mtiles, ntiles, mt, nt, xcd);
    }
  } else {
    tile_of(blockIdx.x, mtiles, ntiles, mt, nt, xcd);
  }
  if (KS == 1 && (int)blockIdx.x >= mtiles * ntiles) return;  // grid padded for split-K
  const int row0 = mt * BM;
  const int col0 = nt * BN;
  if (row0 >= Meff) return;
  const int nk = nk_all / KS;
  const int kt0 = ks * nk;
  if (KS > 1) C = Cpart + (long)ks * ((Meff + BM - 1) / BM) * BM * ldc;
  mac_tile<T, BK, PAD>(A, B, C, M, Meff, row0, col0, kt0, kt0 + nk, lda, ldb, ldc, Nstore, As, Bs);
}

// ---------------------------------------------------------------------------
// Split-BF16 (three products): A = Ah + Al, B = Bh + Bl with bf16 planes,
// C ~= Ah Bh + Ah Bl + Al Bh accumulated in FP32 (v_mfma_f32_16x16x32_bf16,
// gfx950).  Lane layout (16 x 16 x 32): A[i][k] in lane i + 16 (k / 8),
// element k % 8; B[k][j] in lane j + 16 (k / 8), element k % 8; D as above.
// B is stored transposed (Bt[N][K]) so both operands are k-contiguous.
// ---------------------------------------------------------------------------
constexpr int BK16 = 32;
constexpr int PAD16 = 8;  // bf16 elements of row padding in LDS

// One output tile of BMV rows (128, or 64 / 32 for few active rows) over the
// K-tiles [k0, k1), split-BF16.  Two LDS buffers (80 KB: two workgroups fit
// a CU), one barrier per K-tile; the next K-tile waits in registers while the
// current one is multiplied.  Waves 2 x 2, each BMV / 2 rows x 64 columns.
template <int BMV = BM>
__device__ inline void mac_tile_bf16(const __bf16* __restrict__ A, long a_plane,
                                     const __bf16* __restrict__ Bt, long b_plane,
                                     float* __restrict__ C, int M, int Meff, int row0, int col0,
                                     int k0, int k1, long lda, long ldb, long ldc, int Nstore,
                                     __bf16 (&Ash)[2][2][BM][BK16 + PAD16],
                                     __bf16 (&Bsh)[2][2][BN][BK16 + PAD16]) {
  constexpr int IM = BMV / 32;                   // 16-row blocks per wave
  constexpr int AVEC = BMV * (BK16 / 8);         // 16-byte A vectors per plane and K-tile
  constexpr int AV = (AVEC + NTHREADS - 1) / NTHREADS;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave >> 1) * (BMV / 2);
  const int wn0 = (wave & 1) * 64;

  // A: vector e = tid + q 256 is row e / 4, k offset 8 (e % 4); B: each
  // thread moves 16 bf16 (two 16-byte vectors) of one row per plane
  const int g_row = tid >> 1;           // 0..127
  const int g_k = (tid & 1) * 16;       // 0 or 16
  const __bf16* b_src = Bt + (long)(col0 + g_row) * ldb + g_k;

  typedef unsigned int vec_t __attribute__((ext_vector_type(4)));  // 8 bf16 (native vector: stays in registers)
  vec_t ra[2][AV], rb[2][2];  // [plane][vector]
  auto a_row_of = [&](int e) {
    int g = row0 + (e >> 2);
    return g > M - 1 ? M - 1 : g;
  };

  auto gload = [&](int kt) {
    const long off = (long)kt * BK16;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
#pragma unroll
      for (int q = 0; q < AV; ++q) {
        const int e = tid + q * NTHREADS;
        if (AVEC % NTHREADS == 0 || e < AVEC)
          ra[p][q] = *reinterpret_cast<const vec_t*>(A + p * a_plane + (long)a_row_of(e) * lda +
                                                     off + (e & 3) * 8);
      }
      const vec_t* pb = reinterpret_cast<const vec_t*>(b_src + p * b_plane + off);
      rb[p][0] = pb[0];
      rb[p][1] = pb[1];
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
#pragma unroll
      for (int q = 0; q < AV; ++q) {
        const int e = tid + q * NTHREADS;
        if (AVEC % NTHREADS == 0 || e < AVEC)
          *reinterpret_cast<vec_t*>(&Ash[buf][p][e >> 2][(e & 3) * 8]) = ra[p][q];
      }
      vec_t* db = reinterpret_cast<vec_t*>(&Bsh[buf][p][g_row][g_k]);
      db[0] = rb[p][0];
      db[1] = rb[p][1];
    }
  };

  float4_ acc[IM][4];
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = float4_{0, 0, 0, 0};

  gload(k0);
  sstore(0);
  __syncthreads();
  const int lr = lane & 15;
  const int lk = (lane >> 4) * 8;
  for (int kt = k0; kt < k1; ++kt) {
    const int cur = (kt - k0) & 1;
    if (kt + 1 < k1) gload(kt + 1);
    bf16x8_ ah[IM], al[IM], bh[4], bl[4];
#pragma unroll
    for (int i = 0; i < IM; ++i) {
      ah[i] = *reinterpret_cast<const bf16x8_*>(&Ash[cur][0][wm0 + 16 * i + lr][lk]);
      al[i] = *reinterpret_cast<const bf16x8_*>(&Ash[cur][1][wm0 + 16 * i + lr][lk]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bh[j] = *reinterpret_cast<const bf16x8_*>(&Bsh[cur][0][wn0 + 16 * j + lr][lk]);
      bl[j] = *reinterpret_cast<const bf16x8_*>(&Bsh[cur][1][wn0 + 16 * j + lr][lk]);
    }
#pragma unroll
    for (int i = 0; i < IM; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
    if (kt + 1 < k1) sstore(cur ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < IM; ++i) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = row0 + wm0 + 16 * i + (lane >> 4) * 4 + v;
      if (row >= Meff) continue;
      float* crow = C + (long)row * ldc;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = col0 + wn0 + 16 * j + lr;
        if (col < Nstore) crow[col] = acc[i][j][v];
      }
    }
  }
}

__global__ void __launch_bounds__(NTHREADS, 2)
gemm_bf16x3_kernel(const __bf16* __restrict__ A, long a_plane, const __bf16* __restrict__ Bt,
                   long b_plane, float* __restrict__ C, int M, int N, int K, long lda, long ldb,
                   long ldc, int Nstore, const int* __restrict__ M_dev, int m_scale,
                   float* __restrict__ Cpart, int xcd, int streamk) {
  __shared__ __attribute__((aligned(16))) __bf16 Ash[2][2][BM][BK16 + PAD16];  // [buf][plane]
  __shared__ __attribute__((aligned(16))) __bf16 Bsh[2][2][BN][BK16 + PAD16];

  const int mtiles = (M + BM - 1) / BM;
  const int ntiles = N / BN;
  int Meff = M;
  if (M_dev) {
    const int md = M_dev[0] * m_scale;
    Meff = md < M ? md : M;
  }
  const int nk_all = K / BK16;
  if (streamk) {
    const SkPlan p = sk_plan(Meff, ntiles, (int)gridDim.x, nk_all);
    const int v = sk_range_of(blockIdx.x, gridDim.x, xcd);
    long long it, end;
    sk_range(p, v, it, end);
    const long segstride = (long)p.mta * p.bm * ldc;
    while (it < end) {
      int t, k0, k1, s0, ns;
      sk_piece(p, it, end, t, k0, k1);
      sk_segments(p, t, s0, ns);
      float* dst = Cpart + (long)(v - s0) * segstride;
      const int row0 = (t % p.mta) * p.bm, col0 = (t / p.mta) * BN;
      const int hb = sk_tile_height(p, t % p.mta, Meff);
      if (hb == 32)
        mac_tile_bf16<32>(A, a_plane, Bt, b_plane, dst, M, Meff, row0, col0, k0, k1, lda, ldb, ldc,
                          Nstore, Ash, Bsh);
      else if (hb == 64)
        mac_tile_bf16<64>(A, a_plane, Bt, b_plane, dst, M, Meff, row0, col0, k0, k1, lda, ldb, ldc,
                          Nstore, Ash, Bsh);
      else
        mac_tile_bf16(A, a_plane, Bt, b_plane, dst, M, Meff, row0, col0, k0, k1, lda, ldb, ldc,
                      Nstore, Ash, Bsh);
      it += k1 - k0;
    }
    return;
  }
  int mt, nt, ks = 0, KS = 1;
  if (Cpart) {
    const int mta = (Meff + BM - 1) / BM;
    KS = splitk_of(mta, ntiles, (int)gridDim.x, nk_all);
    if (KS > 1) {
      const int tiles = mta * ntiles;
      if ((int)blockIdx.x >= tiles * KS) return;
      const int t = blockIdx.x % tiles;
      ks = blockIdx.x / tiles;
      nt = t / mta;
      mt = t % mta;
    } else {
      tile_of(blockIdx.x, mtiles, ntiles, mt, nt, xcd);
    }
  } else {
    tile_of(blockIdx.x, mtiles, ntiles, mt, nt, xcd);
  }
  if (KS == 1 && (int)blockIdx.x >= mtiles * ntiles) return;  // grid padded for split-K
  const int row0 = mt * BM;
  const int col0 = nt * BN;
  if (row0 >= Meff) return;
  const int nk = nk_all / KS;
  const int kt0 = ks * nk;
  if (KS > 1) C = Cpart + (long)ks * ((Meff + BM - 1) / BM) * BM * ldc;
  mac_tile_bf16(A, a_plane, Bt, b_plane, C, M, Meff, row0, col0, kt0, kt0 + nk, lda, ldb, ldc,
                Nstore, Ash, Bsh);
}

}  // namespace

// Few-row FP64 products (static M <= 8): C[m][c] = sum_k A[m][k] B[k][c] for
// c < Nstore.  One workgroup per 64 output columns and row m; its four
// wavefronts split K and combine through LDS.  Lanes own columns, so every
// load of B is coalesced; the tiled kernel would run a handful of workgroups
// through the whole K loop here.
constexpr int kRowsMax = 8;
__global__ void __launch_bounds__(256) k_gemm_rows64(const double* __restrict__ A, long lda,
                                                     const double* __restrict__ B, long ldb,
                                                     double* __restrict__ C, long ldc, int K,
                                                     int Nstore) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = blockIdx.x * 64 + lane;
  const double* a = A + (long)blockIdx.y * lda;
  const int kc = (K + 3) / 4;
  const int k0 = wave * kc, k1 = min(K, k0 + kc);
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  int k = k0;
  for (; k + 3 < k1; k += 4) {
    acc0 += a[k] * B[(long)k * ldb + col];
    acc1 += a[k + 1] * B[(long)(k + 1) * ldb + col];
    acc2 += a[k + 2] * B[(long)(k + 2) * ldb + col];
    acc3 += a[k + 3] * B[(long)(k + 3) * ldb + col];
  }
  for (; k < k1; ++k) acc0 += a[k] * B[(long)k * ldb + col];
  __shared__ double part[4][64];
  part[wave][lane] = (acc0 + acc1) + (acc2 + acc3);
  __syncthreads();
  if (wave == 0 && col < Nstore)
    C[(long)blockIdx.y * ldc + col] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

void gemm_launch(const GemmArgs& g, hipStream_t s) {
  LYAP_REQUIRE(g.N % BN == 0, LYAP_E_INVAL, "gemm: N not padded");
  LYAP_REQUIRE(g.M >= 1, LYAP_E_INVAL, "gemm: M < 1");
  LYAP_REQUIRE(g.Cpart == nullptr || g.M_dev != nullptr, LYAP_E_INVAL, "gemm: split-K needs M_dev");
  const int mtiles = (int)((g.M + BM - 1) / BM);
  const int ntiles = (int)(g.N / BN);
  const int64_t nblocks = gemm_grid_of(g);
  if (g.streamk) {
    LYAP_REQUIRE(g.M_dev != nullptr && g.Cpart != nullptr && g.grid_min >= 1 &&
                     g.grid_min <= (1 << 20),
                 LYAP_E_INVAL, "gemm: stream-K needs M_dev, Cpart and a grid");
    LYAP_REQUIRE(g.Cpart_rows >= sk_part_rows(g.M, ntiles, (int)g.grid_min, gemm_nk_of(g)),
                 LYAP_E_INVAL, "gemm: stream-K partial buffer too small for the launch");
  } else {
    // split-K writes at most max(mtiles, nblocks / ntiles) row tiles of partials
    LYAP_REQUIRE(g.Cpart == nullptr ||
                     g.Cpart_rows >= std::max<int64_t>(mtiles, nblocks / ntiles) * BM,
                 LYAP_E_INVAL, "gemm: split-K partial buffer too small for the launch");
  }
  dim3 grid((unsigned)nblocks), block(NTHREADS);
  switch (g.type) {
    case GemmType::F64: {
      const int bk = gemm_bk_of(g);
      LYAP_REQUIRE(g.K % bk == 0, LYAP_E_INVAL, "gemm: K not padded");
      if (g.M <= kRowsMax && !g.M_dev && !g.Cpart && !g.tuning && !g.streamk) {
        hipLaunchKernelGGL(k_gemm_rows64, dim3((unsigned)(g.N / 64), (unsigned)g.M), dim3(256), 0, s,
                           (const double*)g.A, (long)g.lda, (const double*)g.B, (long)g.ldb,
                           (double*)g.C, (long)g.ldc, (int)g.K, (int)g.Nstore);
        break;
      }
      auto kern = g.tuning ? (bk == 8 ? gemm_kernel<double, 8, true> : gemm_kernel<double, 16, true>)
                           : (bk == 8 ? gemm_kernel<double, 8> : gemm_kernel<double, 16>);
      hipLaunchKernelGGL(kern, grid, block, 0, s, (const double*)g.A, (const double*)g.B,
                         (double*)g.C, (int)g.M, (int)g.N, (int)g.K, (long)g.lda, (long)g.ldb,
                         (long)g.ldc, (int)g.Nstore, g.M_dev, g.m_scale, (double*)g.Cpart,
                         g.xcd_off ? 0 : 1, g.streamk ? 1 : 0);
      break;
    }
    case GemmType::F32: {
      const int bk = gemm_bk_of(g);
      LYAP_REQUIRE(g.K % bk == 0, LYAP_E_INVAL, "gemm: K not padded");
      auto kern = g.tuning ? (bk == 16 ? gemm_kernel<float, 16, true> : gemm_kernel<float, 32, true>)
                           : (bk == 16 ? gemm_kernel<float, 16> : gemm_kernel<float, 32>);
      hipLaunchKernelGGL(kern, grid, block, 0, s, (const float*)g.A, (const float*)g.B,
                         (float*)g.C, (int)g.M, (int)g.N, (int)g.K, (long)g.lda, (long)g.ldb,
                         (long)g.ldc, (int)g.Nstore, g.M_dev, g.m_scale, (float*)g.Cpart,
                         g.xcd_off ? 0 : 1, g.streamk ? 1 : 0);
      break;
    }
    case GemmType::BF16X3:
      LYAP_REQUIRE(g.K % BK16 == 0, LYAP_E_INVAL, "gemm: K not padded");
      hipLaunchKernelGGL(gemm_bf16x3_kernel, grid, block, 0, s, (const __bf16*)g.A,
                         (long)g.a_plane, (const __bf16*)g.B, (long)g.b_plane, (float*)g.C,
                         (int)g.M, (int)g.N, (int)g.K, (long)g.lda, (long)g.ldb, (long)g.ldc,
                         (int)g.Nstore, g.M_dev, g.m_scale, (float*)g.Cpart, g.xcd_off ? 0 : 1,
                         g.streamk ? 1 : 0);
      break;
  }
  LYAP_HIP(hipGetLastError());
}

}  // namespace lyap
