// The seed Lyapunov solve with a low-rank right-hand side in physical
// coordinates (eq:Z(v) of Section 2.1), and the collapsed trace functional.
//
//   lyap_seed_apply:  G = V^T X,  A0 X + X A0^T = U Y + Y^T U^T
//     transform-in   rho(Y Q0^-T) = Y Tin                       (MFMA GEMM)
//     Cauchy         Gh_a = sum_b Yh_b o K1_ab + sum_b Uh_b o ((Vh_a o Yh_b) L)
//     transform-out  G = rho(Gh) Tout                           (MFMA GEMM)
//   trace_EX:        trace(E X(p)) = t0 + 2 <Gamma^T, Y(p)>
#include "internal.h"

#include <mutex>

// Work area of lyap_seed_apply_noalloc: one copy per GPU, alive until the
// process ends.  Host code never passes this name to a kernel or a copy: it
// stands for the host-side shadow, not the device address.  The device
// address comes from hipGetSymbolAddress, once per device.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace lyap {

namespace {

__device__ inline int us(int u, int h, bool& pr) {
  pr = u < h;
  return pr ? 2 * u : u + h;
}

__global__ void k_apply_formX(double* __restrict__ X, const double* __restrict__ Vh,
                              const double* __restrict__ Yh, int r, int h, int n, int ld) {
  const int row = blockIdx.y;  // (q r + a) r + b
  const int b = row % r, a = (row / r) % r, q = row / (r * r);
  const double* va = Vh + (long)a * ld;
  const double* yb = Yh + ((long)q * r + b) * ld;
  double* xo = X + (long)row * ld;
  for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < n - h; u += gridDim.x * blockDim.x) {
    bool pr;
    const int i = us(u, h, pr);
    if (pr) {
      const double ar = va[i], ai = va[i + 1], br = yb[i], bi = yb[i + 1];
      xo[i] = ar * br - ai * bi;
      xo[i + 1] = ar * bi + ai * br;
    } else {
      xo[i] = va[i] * yb[i];
    }
  }
}

__global__ void k_apply_epilogue(double* __restrict__ Gh, const double* __restrict__ Yh,
                                 const double* __restrict__ H, const double* __restrict__ K1,
                                 const double* __restrict__ Uh, int r, int h, int n, int ld) {
  const int row = blockIdx.y;  // q r + a
  const int a = row % r, q = row / r;
  double* go = Gh + (long)row * ld;
  for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < n - h; u += gridDim.x * blockDim.x) {
    bool pr;
    const int i = us(u, h, pr);
    double sr = 0, si = 0;
    for (int b = 0; b < r; ++b) {
      const double* k = K1 + (long)(a * r + b) * ld;
      const double* yb = Yh + ((long)q * r + b) * ld;
      const double* ub = Uh + (long)b * ld;
      const double* hb = H + ((long)row * r + b) * ld;
      if (pr) {
        sr += yb[i] * k[i] - yb[i + 1] * k[i + 1] + ub[i] * hb[i] - ub[i + 1] * hb[i + 1];
        si += yb[i] * k[i + 1] + yb[i + 1] * k[i] + ub[i] * hb[i + 1] + ub[i + 1] * hb[i];
      } else {
        sr += yb[i] * k[i] + ub[i] * hb[i];
      }
    }
    go[i] = sr;
    if (pr) go[i + 1] = si;
  }
}

__global__ void k_pad_rows(double* __restrict__ dst, long ldd, const double* __restrict__ src,
                           long lds_, int n) {
  const int row = blockIdx.y;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    dst[(long)row * ldd + k] = src[(long)row * lds_ + k];
}

void gemm64(const double* A, long lda, const double* B, long ldb, double* C, long ldc, long M,
            long N, long K, long Nstore, hipStream_t s) {
  GemmArgs g{};
  g.type = GemmType::F64;
  g.A = A;
  g.B = B;
  g.C = C;
  g.M = M;
  g.N = N;
  g.K = K;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.Nstore = Nstore;
  g.M_dev = nullptr;
  g.m_scale = 1;
  gemm_launch(g, s);
}

__global__ void k_zero(double* __restrict__ p, long count) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// Bytes of work area one call needs (pads of every row must start at zero).
size_t apply_work_bytes(const lyap_seed_s* sd, long long batch) {
  const long long r = sd->r, ld = sd->ld;
  const size_t rowb = ld * sizeof(double);
  if (sd->basis == LYAP_BASIS_SCHUR)
    return (size_t)(3 * batch * r) * rowb + (size_t)batch * ld * rowb;
  return (size_t)(3 * batch * r + 2 * batch * r * r) * rowb;
}

void apply_check(long long batch, const double* Y, double* G, int prec) {
  LYAP_REQUIRE(batch >= 1, LYAP_E_INVAL, "batch < 1");
  LYAP_REQUIRE(Y && G, LYAP_E_INVAL, "NULL buffer");
  LYAP_REQUIRE(prec == LYAP_PREC_FP64, LYAP_E_UNSUPPORTED, "lyap_seed_apply: only FP64");
}

// The work: `work` holds at least apply_work_bytes(sd, batch) bytes of device memory.
void apply_core(lyap_seed_s* sd, long long batch, const double* Y, double* G, double* work,
                hipStream_t st) {
  const long long r = sd->r, n = sd->n, ld = sd->ld, h = sd->h;
  const size_t need = apply_work_bytes(sd, batch);
  // pads must be zero: clear the whole area once per call (stream ordered; a fill
  // kernel rather than a memset node, so the call can be captured in a graph)
  hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, st, work, (long)(need / sizeof(double)));
  if (sd->basis == LYAP_BASIS_SCHUR) {
    // Ys = Y Z ; T Xs + Xs T^T = Us Ys + Ys^T Us^T ; G = (Vs^T Xs) Z^T
    const long long rows1 = batch * r;
    double* Yp = work;
    double* Ys = Yp + rows1 * ld;
    double* Gs = Ys + rows1 * ld;
    double* Xs = Gs + rows1 * ld;
    const int ub = (int)std::min<long long>((n + 255) / 256, 64);
    hipLaunchKernelGGL(k_pad_rows, dim3(ub, rows1), dim3(256), 0, st, Yp, (long)ld, Y, (long)n,
                       (int)n);
    gemm64(Yp, ld, sd->Tin.as<double>(), ld, Ys, ld, rows1, ld, ld, ld, st);
    trilyap_launch(sd->T.as<double>(), sd->Tt.as<double>(), Xs, ld * ld, nullptr, 0,
                   sd->Uh.as<double>(), Ys, r * ld, (int)r, (int)n, (int)ld, (int)batch, nullptr,
                   nullptr, st);
    project_launch(sd->Vh.as<double>(), Xs, ld * ld, Gs, r * ld, (int)r, (int)n, (int)ld,
                   (int)batch, nullptr, nullptr, st);
    gemm64(Gs, ld, sd->Tout.as<double>(), ld, G, n, rows1, ld, ld, n, st);
    LYAP_HIP(hipGetLastError());
    return;
  }
  const long long rows1 = batch * r, rows2 = batch * r * r;
  double* Yp = work;
  double* Yh = Yp + rows1 * ld;
  double* Gh = Yh + rows1 * ld;
  double* X = Gh + rows1 * ld;
  double* H = X + rows2 * ld;
  const int ub = (int)std::min<long long>((n + 255) / 256, 64);
  hipLaunchKernelGGL(k_pad_rows, dim3(ub, rows1), dim3(256), 0, st, Yp, (long)ld, Y, (long)n, (int)n);
  gemm64(Yp, ld, sd->Tin.as<double>(), ld, Yh, ld, rows1, ld, ld, ld, st);
  hipLaunchKernelGGL(k_apply_formX, dim3(ub, rows2), dim3(256), 0, st, X, sd->Vh.as<double>(), Yh,
                     (int)r, (int)h, (int)n, (int)ld);
  gemm64(X, ld, sd->Mc.as<double>(), ld, H, ld, rows2, ld, ld, ld, st);
  hipLaunchKernelGGL(k_apply_epilogue, dim3(ub, rows1), dim3(256), 0, st, Gh, Yh, H,
                     sd->K1.as<double>(), sd->Uh.as<double>(), (int)r, (int)h, (int)n, (int)ld);
  gemm64(Gh, ld, sd->Tout.as<double>(), ld, G, n, rows1, ld, ld, n, st);
  LYAP_HIP(hipGetLastError());
}

void apply_impl(lyap_seed_s* sd, long long batch, const double* Y, double* G, int prec,
                hipStream_t st) {
  apply_check(batch, Y, G, prec);
  const size_t need = apply_work_bytes(sd, batch);
  if (sd->scratch_bytes < need) {
    sd->scratch.alloc(need);
    sd->scratch_bytes = need;
  }
  apply_core(sd, batch, Y, G, sd->scratch.as<double>(), st);
}

// Device address of `scratch` on each device, taken once per device with that
// device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

double* noalloc_scratch(int device) {
  LYAP_REQUIRE(device >= 0 && device < kMaxDevices, LYAP_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    LYAP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    LYAP_REQUIRE(p != nullptr, LYAP_E_DEVICE, "no device address for the no-alloc work area");
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  return g_scratch_ptr[device];
}

void apply_noalloc(lyap_seed_s* sd, long long batch, const double* Y, double* G, int prec,
                   hipStream_t st) {
  apply_check(batch, Y, G, prec);
  const size_t need = apply_work_bytes(sd, batch);
  LYAP_REQUIRE(need <= kNoAllocScratchBytes, LYAP_E_INVAL,
               "lyap_seed_apply_noalloc: the batch needs " + std::to_string(need) +
                   " bytes of work area, more than the fixed " +
                   std::to_string(kNoAllocScratchBytes) + "; use a smaller batch");
  int dev = -1;
  LYAP_HIP(hipGetDevice(&dev));
  LYAP_REQUIRE(dev == sd->device, LYAP_E_INVAL,
               "lyap_seed_apply_noalloc: the current device is not the seed's device");
  apply_core(sd, batch, Y, G, noalloc_scratch(dev), st);
}

__global__ void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, long count) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

}  // namespace

// The seed Lyapunov solve with a low-rank right-hand side, FP64, for other
// parts of the library.
void seed_apply64(lyap_seed_s* sd, long long batch, const double* Y, double* G, hipStream_t st) {
  apply_impl(sd, batch, Y, G, LYAP_PREC_FP64, st);
}

}  // namespace lyap

using namespace lyap;


extern "C" {

lyap_status lyap_seed_apply(lyap_seed sd, int64_t batch, const double* Y_dev, double* G_dev,
                            int32_t prec, void* hip_stream) {
  if (!sd) return LYAP_E_INVAL;
  LYAP_TRY(apply_impl(sd, batch, Y_dev, G_dev, prec, (hipStream_t)hip_stream));
  return LYAP_OK;
}

lyap_status lyap_seed_apply_noalloc(lyap_seed sd, int64_t batch, const double* Y_dev,
                                    double* G_dev, int32_t prec, void* hip_stream) {
  if (!sd) return LYAP_E_INVAL;
  LYAP_TRY(apply_noalloc(sd, batch, Y_dev, G_dev, prec, (hipStream_t)hip_stream));
  return LYAP_OK;
}

lyap_status trace_EX(lyap_seed sd, int64_t P, const double* Y_dev, double* trace_dev,
                     void* hip_stream) {
  if (!sd || P < 1 || !Y_dev || !trace_dev) return LYAP_E_INVAL;
  LYAP_TRY(batched_dot(trace_dev, Y_dev, sd->n, sd->Gam.as<double>(), sd->ld, (int)sd->r, (int)P,
                       (int)sd->n, sd->t0, 2.0, (hipStream_t)hip_stream));
  return LYAP_OK;
}

lyap_status lyap_calib_copy(const void* src, void* dst, size_t bytes, void* hip_stream) {
  if (!src || !dst || bytes % 16 != 0) return LYAP_E_INVAL;
  LYAP_TRY({
    const long count = (long)(bytes / 16);
    hipLaunchKernelGGL(k_copy16, dim3(2048), dim3(256), 0, (hipStream_t)hip_stream,
                       (const uint4*)src, (uint4*)dst, count);
    LYAP_HIP(hipGetLastError());
  });
  return LYAP_OK;
}

}  // extern "C"
