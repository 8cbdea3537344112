// Sliding-window form of the stream state (cyc_create_window in
// include/cyclo.h): each committed hop of products keeps its own FP64
// contribution in a ring of n_hops slots instead of being added to one sum;
// a read adds the slots of the window oldest first and re-references the
// phase to the window's first product (the block's `state`, Sec. 4).
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace cyclo {
namespace window {

// ring[(c0 + c) mod W][i] = part[c][i] * E[c][a], c < nc, in ascending c (a
// later hop of the same launch overwrites an earlier one in the same slot).
__global__ void window_store_kernel(double2* ring, const float2* part, const double2* E, int T, int A, int nc,
                                    int64_t c0, int W) {
  const int64_t n2 = 2 * (int64_t)T * A;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n2) return;
  const int a = (int)(i % A);
  for (int c = 0; c < nc; ++c) {
    const float2 p = part[(int64_t)c * n2 + i];
    const double2 e = E[(int64_t)c * A + a];
    const double pr = p.x, pi = p.y;
    ring[((c0 + c) % W) * n2 + i] = make_double2(pr * e.x - pi * e.y, pr * e.y + pi * e.x);
  }
}

__device__ __forceinline__ double frac_prod_w(double alpha, int64_t n) {
  const double nd = (double)n;
  const double p = alpha * nd;
  const double e = fma(alpha, nd, -p);
  double phi = (p - floor(p)) + e;
  phi -= floor(phi);
  return phi >= 1.0 ? 0.0 : phi;
}

// out = (sum_{j < Wn} ring[(s0 + j) mod W]) exp(+j2pi frac(alpha n_ref)) / nd
template <int C128>
__global__ void window_finalize_kernel(const double2* ring, int W, int s0, int Wn, int T, int A,
                                       const double* alpha_r, int64_t n_ref, double nd, void* R, void* Rc) {
  const int64_t TA = (int64_t)T * A;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * TA) return;
  const int table = i >= TA ? 1 : 0;
  void* out = table ? Rc : R;
  if (out == nullptr) return;
  const int64_t r = i - table * TA;
  const int a = (int)(r % A);
  double sr = 0.0, si = 0.0;
  for (int j = 0; j < Wn; ++j) {
    const double2 v = ring[(int64_t)((s0 + j) % W) * 2 * TA + i];
    sr += v.x;
    si += v.y;
  }
  double s, c;
  sincospi(2.0 * frac_prod_w(alpha_r[a], n_ref), &s, &c);  // exp(+j2pi phi) = c + j s
  const double yr = (sr * c - si * s) / nd, yi = (sr * s + si * c) / nd;
  if (C128)
    reinterpret_cast<double2*>(out)[r] = make_double2(yr, yi);
  else
    reinterpret_cast<float2*>(out)[r] = make_float2((float)yr, (float)yi);
}

}  // namespace window

inline unsigned wblocks(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_window_store(double2* ring, const float2* part, const double2* E, int T, int A, int nc,
                               int64_t c0, int W, hipStream_t st) {
  hipLaunchKernelGGL(window::window_store_kernel, dim3(wblocks(2 * (int64_t)T * A)), dim3(256), 0, st, ring, part,
                     E, T, A, nc, c0, W);
  return hipGetLastError();
}

hipError_t launch_window_finalize(const double2* ring, int W, int s0, int Wn, int T, int A, const double* alpha_r,
                                  int64_t n_ref, int64_t n_used, void* R, void* Rc, int c128, hipStream_t st) {
  const int64_t n = 2 * (int64_t)T * A;
  if (c128)
    hipLaunchKernelGGL(window::window_finalize_kernel<1>, dim3(wblocks(n)), dim3(256), 0, st, ring, W, s0, Wn, T, A,
                       alpha_r, n_ref, (double)n_used, R, Rc);
  else
    hipLaunchKernelGGL(window::window_finalize_kernel<0>, dim3(wblocks(n)), dim3(256), 0, st, ring, W, s0, Wn, T, A,
                       alpha_r, n_ref, (double)n_used, R, Rc);
  return hipGetLastError();
}

}  // namespace cyclo
