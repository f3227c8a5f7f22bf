// Shared definitions of the lyapsmw library (device layouts, error plumbing).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstdio>
#include <new>
#include <string>
#include <vector>

#include "../../include/lyapsmw.h"
#include "streamk.h"

namespace lyap {

// Every n-vector on the device is stored with this padded length, zero beyond n,
// so GEMM tiles never need bounds checks along K and N.
constexpr int kPad = 128;
inline int64_t pad_to(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

constexpr int kMaxRestart = 64;
constexpr int kMaxRank = 16;

// Thrown inside the library only; every C entry point catches and converts.
struct Error {
  lyap_status st;
  std::string msg;
};

#define LYAP_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      throw ::lyap::Error{LYAP_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    }                                                                               \
  } while (0)

#define LYAP_REQUIRE(cond, code, text)                 \
  do {                                                 \
    if (!(cond)) throw ::lyap::Error{code, text};      \
  } while (0)

void set_last_error(const std::string& s);

// Wrap the body of a C entry point: library errors become status codes.
#define LYAP_TRY(...)                                   \
  try {                                                 \
    __VA_ARGS__;                                        \
  } catch (const ::lyap::Error& e) {                    \
    ::lyap::set_last_error(e.msg);                      \
    return e.st;                                        \
  } catch (const std::bad_alloc&) {                     \
    ::lyap::set_last_error("host allocation failed");   \
    return LYAP_E_NOMEM;                                \
  } catch (...) {                                       \
    ::lyap::set_last_error("unexpected exception");     \
    return LYAP_E_DEVICE;                               \
  }

// A device allocation owned by RAII.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t b) { alloc(b); }
  void alloc(size_t b) {
    release();
    if (b == 0) return;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      throw Error{LYAP_E_NOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed"};
    }
    bytes = b;
  }
  // a view of memory owned elsewhere (e.g. a caller's workspace): never freed here
  void view(void* ptr, size_t b) {
    release();
    p = ptr;
    bytes = b;
    owned = false;
  }
  void release() {
    if (p && owned) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    owned = true;
  }
  bool owned = true;
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  template <class T> T* as() const { return reinterpret_cast<T*>(p); }
};

// Split-K factor of a dynamic-M GEMM launch: when only a few row tiles are
// active (a tail of the sweep), idle workgroups take K-slices of the same
// tiles; partial products go to a separate buffer and the consumer sums the
// KS slices in fixed order.  Same formula on host and device; at most
// kMaxSplit slices.
constexpr int kMaxSplit = 16;
__host__ __device__ inline int splitk_of(int m_active_tiles, int ntiles, int grid, int nk) {
  const int tiles = m_active_tiles * ntiles;
  if (tiles <= 0) return 1;
  int ks = 1;
  while (ks < kMaxSplit && tiles * ks * 2 <= grid && nk % (ks * 2) == 0 && nk / (ks * 2) >= 4)
    ks *= 2;
  return ks;
}

// Precision of one GEMM launch.
enum class GemmType { F64 = 0, F32 = 1, BF16X3 = 2 };

// C[M x N] = A[M x K] * B[K x N], row-major, K and N multiples of the tile
// (guaranteed by kPad).  Rows >= M (static) or >= *M_dev (dynamic, if given)
// are neither read beyond the clamp nor stored.  Columns >= Nstore not stored.
// F64: A, B, C double.  F32: A, B float, C float.
// BF16X3: A and B given as (hi, lo) bf16 pairs; B stored transposed (N x K);
//         C float.
struct GemmArgs {
  GemmType type;
  const void* A;      // F64/F32: M x lda ; BF16X3: hi plane, lo plane at A + a_plane
  const void* B;      // F64/F32: K x ldb ; BF16X3: Bt hi (N x ldb), lo at B + b_plane
  void* C;
  int64_t M, N, K;
  int64_t lda, ldb, ldc;
  int64_t Nstore;     // columns actually written
  int64_t a_plane, b_plane;  // element offsets of the lo planes (BF16X3)
  const int* M_dev;   // optional device row count (scaled by m_scale)
  int m_scale;
  void* Cpart;        // optional split-K partial buffer, dynamic M only (size: see grid_min)
  int64_t grid_min;   // optional: launch at least this many workgroups (more split-K
                      // slices for skinny shapes); Cpart must hold
                      // max(row tiles, grid / column tiles) row tiles of ldc
  int64_t Cpart_rows; // rows (of ldc elements) that Cpart holds; checked before launch
  int bk;             // K-tile depth (0: the type's default; F64 8 or 16, F32 16 or 32)
  int xcd_off;        // 1: plain tile order instead of the XCD-aware mapping
  int tuning;         // 1: autotuner timing launch (separate kernel symbol)
  int streamk;        // 1: stream-K (dynamic M, Cpart holds segments; C is not
                      // written): exactly grid_min workgroups, see sk_plan
};

inline int gemm_bk(GemmType t) { return t == GemmType::F64 ? 16 : 32; }
inline int gemm_bk_of(const GemmArgs& g) { return g.bk > 0 ? g.bk : gemm_bk(g.type); }
// K-tiles of one launch (the BF16X3 kernel's K-tile is 32)
inline int gemm_nk_of(const GemmArgs& g) {
  return (int)(g.K / (g.type == GemmType::BF16X3 ? 32 : gemm_bk_of(g)));
}
// workgroups of a launch (the consumer of split-K or stream-K partials needs it)
inline int64_t gemm_grid_of(const GemmArgs& g) {
  if (g.streamk) return g.grid_min;
  const int64_t tiles = ((g.M + kGemmBM - 1) / kGemmBM) * (g.N / kGemmBN);
  return tiles > g.grid_min ? tiles : g.grid_min;
}

void gemm_launch(const GemmArgs& g, hipStream_t s);

}  // namespace lyap
