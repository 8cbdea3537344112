// Cyclic spectrum from a lag table (cyc_scf in include/cyclo.h): the cyclic
// Wiener-Khinchin relation, spectral analysis the paper leaves for future work
// (Sec. 6):
//   S[k][a] = sum_t w(m_t) exp(-j pi alpha_a m_t) R[t][a] exp(-j2pi f_k m_t),
//   m_t = lag_min + t, f_k = -1/2 + k / F.
// Pass 1 forms P[t][a] = w(m_t) exp(-j pi alpha_a m_t) R[t][a] (the phase in
// FP64 from an error-free reduction); pass 2 is the lag DFT, one thread per
// (f_k, alpha), with the twiddles exp(-j2pi f_k m) of a workgroup's frequency
// staged in LDS (the angle f_k m mod 1 is an exact rational).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "../../include/cyclo.h"

namespace cyclo {
namespace scf {

constexpr int MAX_LAGS = 8192;

__device__ __forceinline__ double frac_half(double alpha, int64_t m) {
  // frac(alpha * m / 2) with an error-free product (|alpha| and |m| bounded)
  const double md = 0.5 * (double)m;
  const double p = alpha * md;
  const double e = fma(alpha, md, -p);
  double phi = (p - floor(p)) + e;
  phi -= floor(phi);
  return phi >= 1.0 ? 0.0 : phi;
}

__global__ void scf_weight_kernel(const float2* R, const double* alphas, int A, int64_t lag_min, int T, int window,
                                  float2* P) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)T * A) return;
  const int t = (int)(i / A), a = (int)(i % A);
  const int64_t m = lag_min + t;
  double w = 1.0;
  if (window == 1) {
    const int64_t last = lag_min + T - 1;
    const int64_t M = std::max(lag_min < 0 ? -lag_min : lag_min, last < 0 ? -last : last);
    w = 0.5 * (1.0 + cospi((double)m / (double)(M + 1)));
  }
  double s, c;
  sincospi(2.0 * frac_half(alphas[a], m), &s, &c);  // exp(-j pi alpha m) = c - j s
  const float2 r = R[i];
  P[i] = make_float2((float)(w * ((double)r.x * c + (double)r.y * s)), (float)(w * ((double)r.y * c - (double)r.x * s)));
}

__global__ __launch_bounds__(256) void scf_dft_kernel(const float2* P, int A, int64_t lag_min, int T, int F,
                                                      float2* S) {
  __shared__ float2 tw[MAX_LAGS];
  const int k = blockIdx.y;
  // exp(-j2pi f_k m), f_k m = (k - F/2) m / F: reduce the integer numerator mod F
  for (int t = threadIdx.x; t < T; t += 256) {
    const int64_t m = lag_min + t;
    int64_t num = ((int64_t)(2 * k - F) * m) % (2 * (int64_t)F);  // angle = num / (2F) turns
    if (num < 0) num += 2 * (int64_t)F;
    double s, c;
    sincospi((double)num / (double)F, &s, &c);
    tw[t] = make_float2((float)c, (float)-s);
  }
  __syncthreads();
  const int a = blockIdx.x * 256 + threadIdx.x;
  if (a >= A) return;
  float re = 0.f, im = 0.f;
  for (int t = 0; t < T; ++t) {
    const float2 p = P[(int64_t)t * A + a], e = tw[t];
    re = fmaf(p.x, e.x, fmaf(-p.y, e.y, re));
    im = fmaf(p.x, e.y, fmaf(p.y, e.x, im));
  }
  S[(int64_t)k * A + a] = make_float2(re, im);
}

// Weighted-table workspace of cyc_scf_noalloc: a fixed device array (each GPU
// holds its own copy for the life of the process).  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the symbol);
// it passes the device address that hipGetSymbolAddress returns for the
// current device.
constexpr int64_t NOALLOC_MAX = int64_t(1) << 21;  // weighted-table entries (16 MiB)
static __device__ __align__(256) float2 scratch[NOALLOC_MAX];

constexpr int MAX_DEVICES = 64;

// Device address of `scratch` on the current device, looked up once per device.
float2* scratch_ptr() {
  static std::mutex mu;
  static float2* ptr[MAX_DEVICES] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    ptr[dev] = static_cast<float2*>(p);
  }
  return ptr[dev];
}

bool scf_args_ok(const void* d_R, const double* d_alphas, int32_t n_alpha, int64_t lag_min, int32_t n_lag,
                 int32_t n_freq, int32_t window, const void* d_S) {
  return d_R && d_alphas && d_S && n_alpha >= 1 && n_lag >= 1 && n_lag <= MAX_LAGS && n_freq >= 1 &&
         n_freq <= 65536 && (window == 0 || window == 1) && lag_min >= -(1 << 20) && lag_min <= (1 << 20);
}

int scf_launch(const void* d_R, const double* d_alphas, int32_t n_alpha, int64_t lag_min, int32_t n_lag,
               int32_t n_freq, int32_t window, void* d_S, float2* P, hipStream_t st) {
  const int64_t TA = (int64_t)n_lag * n_alpha;
  hipLaunchKernelGGL(scf_weight_kernel, dim3((unsigned)((TA + 255) / 256)), dim3(256), 0, st,
                     reinterpret_cast<const float2*>(d_R), d_alphas, n_alpha, lag_min, n_lag, window, P);
  hipLaunchKernelGGL(scf_dft_kernel, dim3((unsigned)((n_alpha + 255) / 256), (unsigned)n_freq), dim3(256), 0, st, P,
                     n_alpha, lag_min, n_lag, n_freq, reinterpret_cast<float2*>(d_S));
  return hipGetLastError() == hipSuccess ? CYC_OK : CYC_EDEVICE;
}

}  // namespace scf
}  // namespace cyclo

using namespace cyclo::scf;

extern "C" {

int cyc_scf(const void* d_R, const double* d_alphas, int32_t n_alpha, int64_t lag_min, int32_t n_lag,
            int32_t n_freq, int32_t window, void* d_S, void* stream) {
  if (!scf_args_ok(d_R, d_alphas, n_alpha, lag_min, n_lag, n_freq, window, d_S)) return CYC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t TA = (int64_t)n_lag * n_alpha;
  float2* P = nullptr;
  if (hipMallocAsync(reinterpret_cast<void**>(&P), sizeof(float2) * TA, st) != hipSuccess) return CYC_ENOMEM;
  const int rc = scf_launch(d_R, d_alphas, n_alpha, lag_min, n_lag, n_freq, window, d_S, P, st);
  (void)hipFreeAsync(P, st);
  return rc;
}

int cyc_scf_noalloc(const void* d_R, const double* d_alphas, int32_t n_alpha, int64_t lag_min, int32_t n_lag,
                    int32_t n_freq, int32_t window, void* d_S, void* stream) {
  if (!scf_args_ok(d_R, d_alphas, n_alpha, lag_min, n_lag, n_freq, window, d_S)) return CYC_EINVAL;
  if ((int64_t)n_lag * n_alpha > NOALLOC_MAX) return CYC_EUNSUPPORTED;
  float2* P = scratch_ptr();
  if (!P) return CYC_EDEVICE;
  return scf_launch(d_R, d_alphas, n_alpha, lag_min, n_lag, n_freq, window, d_S, P,
                    reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
