// Cycle-frequency estimation from the cyclic tables (cyc_cfe_* in
// include/cyclo.h).  The paper leaves estimating the cycle frequencies for
// future work (Sec. 6) and names coarse-to-fine searches among related
// estimators (Sec. 1); this is one on the tables of Sec. 4, Eq. (11):
//
//  1. noise scale sigma[t][c] per lag and block c of 64 bins: the median of
//     |R[t][.]| over blocks c-1, c, c+1 (circular), divided by sqrt(2 ln 2)
//     (Rayleigh scale of cells without a feature);
//  2. statistic q[k] = max_t |R[t][k]| / sigma[t][k / 64];
//  3. candidates: q[k] > kappa, q[k] > q[k-1], q[k] >= q[k+1] (circular);
//  4. leakage masking, strongest first: a candidate is kept if at some lag it
//     exceeds kappa sigma and |R[t][k]| > (pi/2) A / (N (d - 1/2)) |R[t][p]|
//     for every kept p at circular distance d (twice the most a feature within
//     half a bin of p leaks through the Dirichlet kernel of N products);
//  5. refinement: the zoom table on alpha_k + (j - Z) / (Z A), j <= 2Z, and
//     the column with the largest max_t |R| / sigma (first of equal ones).
// Magnitudes are sqrt(Re^2 + Im^2) in FP64 and every comparison is FP64, with
// no contraction of the FP64 arithmetic, so decisions on one table are
// reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/cyclo.h"

#pragma clang fp contract(off)

namespace cyclo {
namespace cfe {

constexpr int BLOCK = 64;
constexpr int WIN = 3 * BLOCK;                     // values behind one scale
constexpr int MAXC = 4096;                         // candidates handled per table
constexpr int MAXT = 4096;                         // lags
constexpr double SQRT_2LN2 = 1.1774100225154747;   // sqrt(2 ln 2)
constexpr double HALF_PI = 1.5707963267948966;     // pi / 2

__device__ __forceinline__ double mag(float2 v) {
  const double re = v.x, im = v.y;
  return sqrt(re * re + im * im);
}

// sigma[t][c]: one wave per (t, c); the two middle values of the 192 window
// magnitudes by rank counting (rank = smaller values + equal values earlier in
// the window), then their mean over sqrt(2 ln 2).
__global__ __launch_bounds__(64) void cfe_sigma_kernel(const float2* R, int A, double* sigma) {
  __shared__ double w[WIN];
  const int nb = A / BLOCK;
  const int c = blockIdx.x, t = blockIdx.y, lane = threadIdx.x;
  const float2* row = R + (int64_t)t * A;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int blk = (c + i - 1 + nb) % nb;
    w[i * BLOCK + lane] = mag(row[blk * BLOCK + lane]);
  }
  __syncthreads();
  double lo = 0.0, hi = 0.0;
  int have = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int e = i * BLOCK + lane;
    const double v = w[e];
    int rank = 0;
    for (int f = 0; f < WIN; ++f) {
      const double u = w[f];
      rank += (u < v || (u == v && f < e)) ? 1 : 0;
    }
    if (rank == WIN / 2 - 1) {
      lo = v;
      have |= 1;
    }
    if (rank == WIN / 2) {
      hi = v;
      have |= 2;
    }
  }
  // exactly one lane holds each middle value
  __shared__ double mid[2];
  if (have & 1) mid[0] = lo;
  if (have & 2) mid[1] = hi;
  __syncthreads();
  if (lane == 0) sigma[(int64_t)t * nb + c] = ((mid[0] + mid[1]) * 0.5) / SQRT_2LN2;
}

__device__ __forceinline__ double ratio(double m, double s) {
  const double r = m / s;
  return r != r ? 0.0 : r;  // 0/0 -> 0; m/0 -> inf
}

// q[k] = max_t |R[t][k]| / sigma[t][k / 64]
__global__ __launch_bounds__(256) void cfe_stat_kernel(const float2* R, int T, int A, const double* sigma,
                                                       double* q) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= A) return;
  const int nb = A / BLOCK, c = k / BLOCK;
  double best = 0.0;
  for (int t = 0; t < T; ++t) best = fmax(best, ratio(mag(R[(int64_t)t * A + k]), sigma[(int64_t)t * nb + c]));
  q[k] = best;
}

__device__ __forceinline__ double leak_factor(int d, int A, int64_t N) {
  return HALF_PI * ((double)A / ((double)N * ((double)d - 0.5)));
}

// One workgroup: candidates, masking (strongest first) and the ascending list
// of kept bins other than `exclude`.  status: 0 ok, 1 too many candidates.
__global__ __launch_bounds__(1024) void cfe_detect_kernel(const float2* R, int T, int A, int64_t N,
                                                          const double* sigma, const double* q, double kappa,
                                                          int exclude, int max_out, int32_t* bins,
                                                          int32_t* count, int32_t* status) {
  __shared__ double cq[MAXC];
  __shared__ int ck[MAXC];
  __shared__ int kept[MAXC];
  __shared__ int ncand, nkept;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nb = A / BLOCK;
  if (tid == 0) {
    ncand = 0;
    nkept = 0;
  }
  __syncthreads();
  for (int k = tid; k < A; k += nt) {
    const double v = q[k];
    const double l = q[(k - 1 + A) % A], r = q[(k + 1) % A];
    if (v > kappa && (A == 1 || (v > l && v >= r))) {
      const int slot = atomicAdd(&ncand, 1);
      if (slot < MAXC) {
        cq[slot] = v;
        ck[slot] = k;
      }
    }
  }
  __syncthreads();
  const int nc = ncand;
  if (nc > MAXC) {
    if (tid == 0) {
      *status = 1;
      *count = 0;
    }
    return;
  }
  // bitonic sort of the candidates by (q descending, k ascending), padded
  int P = 1;
  while (P < nc) P <<= 1;
  for (int i = nc + tid; i < P; i += nt) {
    cq[i] = -1.0;
    ck[i] = 0x7fffffff;
  }
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < P; i += nt) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          // "before" = stronger, or equally strong with the lower bin
          const bool jb = cq[j] > cq[i] || (cq[j] == cq[i] && ck[j] < ck[i]);
          if (jb == up) {
            const double tq = cq[i];
            cq[i] = cq[j];
            cq[j] = tq;
            const int tk = ck[i];
            ck[i] = ck[j];
            ck[j] = tk;
          }
        }
      }
      __syncthreads();
    }
  }
  // masking in that order
  for (int i = 0; i < nc; ++i) {
    const int k = ck[i];
    const int c = k / BLOCK;
    const int nk = nkept;
    int ok = 0;
    for (int t = tid; t < T; t += nt) {
      const double m = mag(R[(int64_t)t * A + k]);
      if (!(ratio(m, sigma[(int64_t)t * nb + c]) > kappa)) continue;
      bool clear = true;
      for (int e = 0; e < nk && clear; ++e) {
        const int p = kept[e];
        int d = k > p ? k - p : p - k;
        d = min(d, A - d);
        clear = m > leak_factor(d, A, N) * mag(R[(int64_t)t * A + p]);
      }
      if (clear) ok = 1;
    }
    ok = __syncthreads_or(ok);
    if (ok && tid == 0) kept[nkept++] = k;
    __syncthreads();
  }
  // ascending output without `exclude`
  const int nk = nkept;
  for (int i = tid; i < nk; i += nt) {
    const int k = kept[i];
    if (k == exclude) continue;
    int pos = 0;
    for (int e = 0; e < nk; ++e) {
      const int o = kept[e];
      pos += (o != exclude && o < k) ? 1 : 0;
    }
    if (pos < max_out) bins[pos] = k;
  }
  int found = 0;
  for (int i = tid; i < nk; i += nt) found |= kept[i] == exclude ? 1 : 0;
  found = __syncthreads_or(found);
  if (tid == 0) {
    *count = nk - found;
    *status = 0;
  }
}

// Per peak p: zoom columns [p W, (p+1) W), W = 2Z + 1, of Rz [T][n_peaks W];
// the first column with the largest max_t |Rz| / sigma[t][bins[p] / 64].
__global__ __launch_bounds__(256) void cfe_refine_kernel(const float2* Rz, int T, int n_peaks, int W, int nb,
                                                         const int32_t* bins, const double* sigma, int32_t* jout,
                                                         double* qout) {
  __shared__ double bq[256];
  __shared__ int bj[256];
  const int p = blockIdx.x, tid = threadIdx.x;
  const int c = bins[p] / BLOCK;
  const int64_t cols = (int64_t)n_peaks * W;
  double best = -1.0;
  int bestj = 0x7fffffff;
  for (int j = tid; j < W; j += 256) {
    double v = 0.0;
    for (int t = 0; t < T; ++t) v = fmax(v, ratio(mag(Rz[(int64_t)t * cols + (int64_t)p * W + j]), sigma[(int64_t)t * nb + c]));
    if (v > best || (v == best && j < bestj)) {
      best = v;
      bestj = j;
    }
  }
  bq[tid] = best;
  bj[tid] = bestj;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      const double ov = bq[tid + s];
      const int oj = bj[tid + s];
      if (ov > bq[tid] || (ov == bq[tid] && oj < bj[tid])) {
        bq[tid] = ov;
        bj[tid] = oj;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    jout[p] = bj[0];
    qout[p] = bq[0];
  }
}

int detect_launch(const float2* R, int T, int A, int64_t N, double kappa, int exclude, int max_out, int32_t* bins,
                  int32_t* count, double* sigma, double* q, int32_t* status, hipStream_t st) {
  const int nb = A / BLOCK;
  hipLaunchKernelGGL(cfe_sigma_kernel, dim3(nb, T), dim3(64), 0, st, R, A, sigma);
  hipLaunchKernelGGL(cfe_stat_kernel, dim3((A + 255) / 256), dim3(256), 0, st, R, T, A, sigma, q);
  hipLaunchKernelGGL(cfe_detect_kernel, dim3(1), dim3(1024), 0, st, R, T, A, N, sigma, q, kappa, exclude, max_out,
                     bins, count, status);
  return hipGetLastError() == hipSuccess ? CYC_OK : CYC_EDEVICE;
}

bool detect_args_ok(const void* d_R, int32_t n_lag, int32_t n_alpha, int64_t n_used, double kappa,
                    int32_t exclude_bin, int32_t max_out) {
  return d_R && n_lag >= 1 && n_lag <= MAXT && n_alpha >= BLOCK && n_alpha % BLOCK == 0 && n_used >= 1 &&
         n_used <= n_alpha && std::isfinite(kappa) && kappa >= 0.0 && exclude_bin >= -1 &&
         exclude_bin < n_alpha && max_out >= 0;
}

template <typename T>
hipError_t dalloc(T** p, int64_t n, hipStream_t st) {
  return hipMallocAsync(reinterpret_cast<void**>(p), sizeof(T) * (size_t)std::max<int64_t>(n, 1), st);
}

}  // namespace cfe
}  // namespace cyclo

using namespace cyclo::cfe;

extern "C" {

int cyc_cfe_detect(const void* d_R, int32_t n_lag, int32_t n_alpha, int64_t n_used, double kappa,
                   int32_t exclude_bin, int32_t max_out, int32_t* d_bins, int32_t* d_count, double* d_sigma,
                   void* stream) {
  if (!detect_args_ok(d_R, n_lag, n_alpha, n_used, kappa, exclude_bin, max_out) || !d_count || !d_sigma ||
      (max_out > 0 && !d_bins))
    return CYC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  double* q = nullptr;
  int32_t* status = nullptr;
  if (dalloc(&q, n_alpha, st) != hipSuccess) return CYC_ENOMEM;
  if (dalloc(&status, 1, st) != hipSuccess) {
    (void)hipFreeAsync(q, st);
    return CYC_ENOMEM;
  }
  int rc = detect_launch(reinterpret_cast<const float2*>(d_R), n_lag, n_alpha, n_used, kappa, exclude_bin, max_out,
                         d_bins, d_count, d_sigma, q, status, st);
  int32_t h_status = 0;
  if (rc == CYC_OK && (hipMemcpyAsync(&h_status, status, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
                       hipStreamSynchronize(st) != hipSuccess))
    rc = CYC_EDEVICE;
  (void)hipFreeAsync(q, st);
  (void)hipFreeAsync(status, st);
  if (rc == CYC_OK && h_status != 0) rc = CYC_EUNSUPPORTED;
  return rc;
}

int cyc_cfe_refine(const void* d_Rz, int32_t n_lag, int32_t n_peaks, int32_t zoom, const int32_t* d_bins,
                   const double* d_sigma, int32_t n_alpha, int32_t* d_j, double* d_q, void* stream) {
  if (!d_Rz || !d_bins || !d_sigma || !d_j || !d_q || n_lag < 1 || n_lag > MAXT || n_peaks < 1 || zoom < 1 ||
      zoom > 4096 || n_alpha < BLOCK || n_alpha % BLOCK)
    return CYC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(cfe_refine_kernel, dim3(n_peaks), dim3(256), 0, st, reinterpret_cast<const float2*>(d_Rz), n_lag,
                     n_peaks, 2 * zoom + 1, n_alpha / BLOCK, d_bins, d_sigma, d_j, d_q);
  return hipGetLastError() == hipSuccess ? CYC_OK : CYC_EDEVICE;
}

int cyc_estimate_cycle_freqs(const void* d_x, int64_t n, double alpha0, int32_t n_alpha, int32_t n_lag,
                             int32_t table, double kappa, int32_t zoom, int32_t exclude_zero, int32_t max_out,
                             double* alpha_hat, double* stat, int32_t* bins, int32_t* count, void* stream) {
  if (!d_x || !count || n < 1 || !std::isfinite(alpha0) || (table != 0 && table != 1) || zoom < 1 || zoom > 4096 ||
      max_out < 0 || (max_out > 0 && (!alpha_hat || !stat || !bins)))
    return CYC_EINVAL;
  const int64_t N = n - n_lag + 1;
  if (!detect_args_ok(d_x, n_lag, n_alpha, N, kappa, -1, max_out)) return CYC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int A = n_alpha, T = n_lag;
  const int64_t TA = (int64_t)T * A;
  // the alpha = 0 bin of the non-conjugate table, if it is on the grid
  int exclude = -1;
  if (exclude_zero && table == 0) {
    const double kz = std::nearbyint(-alpha0 * A);
    const int k = (int)(((int64_t)kz % A + A) % A);
    const double a = alpha0 + (double)k / (double)A;
    if (std::fabs(a - std::nearbyint(a)) < 1e-12) exclude = k;
  }
  float2* tab = nullptr;
  double* sigma = nullptr;
  double* q = nullptr;
  int32_t *d_bins = nullptr, *d_meta = nullptr;  // meta: count, status
  int rc = CYC_OK;
  if (dalloc(&tab, TA, st) != hipSuccess || dalloc(&sigma, (int64_t)T * (A / BLOCK), st) != hipSuccess ||
      dalloc(&q, A, st) != hipSuccess || dalloc(&d_bins, std::max(max_out, 1), st) != hipSuccess ||
      dalloc(&d_meta, 2, st) != hipSuccess)
    rc = CYC_ENOMEM;
  // coarse table: the exact uniform-grid form when A is a power of two it
  // supports, else the dense contraction on the grid
  if (rc == CYC_OK) {
    std::vector<double> grid;
    const bool pow2 = (A & (A - 1)) == 0 && A <= 65536;
    int64_t nu = 0;
    if (pow2) {
      cyc_grid* g = nullptr;
      rc = cyc_grid_create(&g, alpha0, A, T, 0, stream);
      if (rc == CYC_OK) rc = cyc_grid_push(g, d_x, n, stream);
      if (rc == CYC_OK) rc = cyc_grid_read(g, table == 0 ? tab : nullptr, table == 1 ? tab : nullptr, &nu, stream);
      if (g) {
        (void)hipStreamSynchronize(st);
        cyc_grid_destroy(g);
      }
    } else {
      grid.resize(A);
      for (int k = 0; k < A; ++k) grid[k] = alpha0 + (double)k / (double)A;
      cyc_state* s = nullptr;
      rc = cyc_create(&s, grid.data(), A, T, 0, stream);
      if (rc == CYC_OK) rc = cyc_push(s, d_x, n, stream);
      if (rc == CYC_OK) rc = cyc_read(s, table == 0 ? tab : nullptr, table == 1 ? tab : nullptr, &nu, stream);
      if (s) {
        (void)hipStreamSynchronize(st);
        cyc_destroy(s);
      }
    }
    if (rc == CYC_OK && nu != N) rc = CYC_EDEVICE;
  }
  if (rc == CYC_OK)
    rc = detect_launch(tab, T, A, N, kappa, exclude, max_out, d_bins, d_meta, sigma, q, d_meta + 1, st);
  int32_t meta[2] = {0, 0};
  if (rc == CYC_OK && (hipMemcpyAsync(meta, d_meta, sizeof(meta), hipMemcpyDeviceToHost, st) != hipSuccess ||
                       hipStreamSynchronize(st) != hipSuccess))
    rc = CYC_EDEVICE;
  if (rc == CYC_OK && meta[1] != 0) rc = CYC_EUNSUPPORTED;
  const int P = rc == CYC_OK ? std::min(meta[0], max_out) : 0;
  if (rc == CYC_OK) *count = meta[0];
  if (rc == CYC_OK && P > 0) {
    std::vector<int32_t> hb(P);
    rc = hipMemcpy(hb.data(), d_bins, sizeof(int32_t) * P, hipMemcpyDeviceToHost) == hipSuccess ? CYC_OK
                                                                                                : CYC_EDEVICE;
    // zoom grid of every detection: alpha_k + (j - Z) / (Z A)
    const int W = 2 * zoom + 1;
    std::vector<double> zg((size_t)P * W);
    for (int p = 0; p < P && rc == CYC_OK; ++p) {
      const double ak = alpha0 + (double)hb[p] / (double)A;
      for (int j = 0; j < W; ++j) zg[(size_t)p * W + j] = ak + (double)(j - zoom) / (double)((int64_t)zoom * A);
    }
    float2* tz = nullptr;
    int32_t* dj = nullptr;
    double* dq = nullptr;
    if (rc == CYC_OK && (dalloc(&tz, (int64_t)T * P * W, st) != hipSuccess || dalloc(&dj, P, st) != hipSuccess ||
                         dalloc(&dq, P, st) != hipSuccess))
      rc = CYC_ENOMEM;
    cyc_state* s = nullptr;
    int64_t nu = 0;
    if (rc == CYC_OK) rc = cyc_create(&s, zg.data(), P * W, T, 0, stream);
    if (rc == CYC_OK) rc = cyc_push(s, d_x, n, stream);
    if (rc == CYC_OK) rc = cyc_read(s, table == 0 ? tz : nullptr, table == 1 ? tz : nullptr, &nu, stream);
    if (rc == CYC_OK) rc = cyc_cfe_refine(tz, T, P, zoom, d_bins, sigma, A, dj, dq, stream);
    std::vector<int32_t> hj(P);
    if (rc == CYC_OK &&
        (hipMemcpyAsync(hj.data(), dj, sizeof(int32_t) * P, hipMemcpyDeviceToHost, st) != hipSuccess ||
         hipMemcpyAsync(stat, dq, sizeof(double) * P, hipMemcpyDeviceToHost, st) != hipSuccess ||
         hipStreamSynchronize(st) != hipSuccess))
      rc = CYC_EDEVICE;
    if (s) {
      (void)hipStreamSynchronize(st);
      cyc_destroy(s);
    }
    if (rc == CYC_OK)
      for (int p = 0; p < P; ++p) {
        bins[p] = hb[p];
        alpha_hat[p] = zg[(size_t)p * W + hj[p]];
      }
    (void)hipFreeAsync(tz, st);
    (void)hipFreeAsync(dj, st);
    (void)hipFreeAsync(dq, st);
  }
  (void)hipFreeAsync(tab, st);
  (void)hipFreeAsync(sigma, st);
  (void)hipFreeAsync(q, st);
  (void)hipFreeAsync(d_bins, st);
  (void)hipFreeAsync(d_meta, st);
  (void)hipStreamSynchronize(st);
  return rc;
}

}  // extern "C"
