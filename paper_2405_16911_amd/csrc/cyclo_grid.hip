// Uniform-grid form (cyc_grid_* in include/cyclo.h): the tables on the whole
// grid alpha_k = alpha0 + k/A by folding and one FFT per lag (the paper's Full
// mode, Sec. 4, evaluates every cycle frequency on a grid with an FFT).
//
// With p_t[n] = x[n+t] conj(x[n]) (or x[n+t] x[n]) and E(n) =
// exp(-j2pi frac(alpha0 n)), the identity exp(-j2pi k n / A) =
// exp(-j2pi k (n mod A) / A) gives
//   S[t][k] = sum_{r<A} exp(-j2pi k r / A) q_t[r],
//   q_t[r]  = sum_{n = r mod A} p_t[n] E(n),
// so a push only adds each product into its fold bin r = n mod A (FP64, in
// ascending n, so any segmentation of the record gives the same bits) and a
// read takes an A-point DFT of every fold row.
//
// HBM layout of one state:
//   q [2][T][A]      FP64 complex fold bins (R rows, then Rc rows)
//   Y [2][T][A]      FP64 complex FFT workspace (A > 8192 only)
//   tw [A]           FP64 twiddles exp(-j2pi i / A)
//   E [maxp]         FP64 complex phases of one launch's products
//   pend[2][T]       pending samples (ping-pong)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>

#include "../../include/cyclo.h"
#include "cyclo_internal.h"

namespace cyclo {
namespace grid {

constexpr int FFT_MAX = 8192;   // largest FFT done in LDS (128 KiB of FP64 complex)
constexpr int FOLD_TT = 8;      // lags per fold thread (fewer when that leaves the GPU short of waves)
constexpr int FOLD_NT = 256;    // threads (fold bins) per fold workgroup
constexpr int64_t MAXP = 1 << 20;  // products folded per launch

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

// frac(alpha * n) in [0, 1) with an error-free product (as the contraction's
// twiddle generator).
__device__ __forceinline__ double frac_mul(double alpha, int64_t n) {
  const double nd = (double)n;
  const double p = alpha * nd;
  const double e = fma(alpha, nd, -p);
  double phi = (p - floor(p)) + e;
  phi -= floor(phi);
  return phi >= 1.0 ? 0.0 : phi;
}

// E[i] = exp(-j2pi frac(alpha0 (n0 + i))), i < np.
__global__ void grid_phase_kernel(double alpha0, int64_t n0, int64_t np, double2* E) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  double s, c;
  sincospi(2.0 * frac_mul(alpha0, n0 + i), &s, &c);
  E[i] = make_double2(c, -s);
}

// Samples of the virtual array pend[0..n_pend) ++ xin (absolute index base + g).
__device__ __forceinline__ float2 gload(const VSrc& v, int64_t g) {
  if (g >= v.n_avail) return make_float2(0.f, 0.f);
  return g < v.n_pend ? v.pend[g] : v.xin[g - v.n_pend];
}

// One thread per (fold bin r, group of TT lags): q[tab][t][r] += p_t[i] E[i]
// for the products i < np whose phase index n0 + i is r (mod A), in ascending i.
// Product i pairs the leading samples vx[i + t] with the trailing sample vy[i]
// (the same array for one input); E[i] is its phase.  Each (bin, lag) sum
// takes the same operations in the same order for any TT.
template <int TT>
__global__ __launch_bounds__(FOLD_NT) void grid_fold_kernel(VSrc vx, VSrc vy, int64_t n0, int64_t np,
                                                             const double2* E, int T, int A, double2* q) {
  const int r = blockIdx.x * FOLD_NT + threadIdx.x;
  const int t0 = blockIdx.y * TT;
  if (r >= A) return;
  const int nt = min(TT, T - t0);
  // first product index i >= 0 with (n0 + i) mod A == r
  const int64_t rem = (int64_t)((n0 % A + A) % A);
  int64_t i = ((int64_t)r - rem) % A;
  if (i < 0) i += A;
  double2 acc[2][TT];
#pragma unroll
  for (int k = 0; k < TT; ++k) {
    acc[0][k] = make_double2(0.0, 0.0);
    acc[1][k] = make_double2(0.0, 0.0);
    if (k < nt) {
      acc[0][k] = q[((int64_t)0 * T + t0 + k) * A + r];
      acc[1][k] = q[((int64_t)1 * T + t0 + k) * A + r];
    }
  }
  for (; i < np; i += A) {
    const float2 x0 = gload(vy, i);
    const double2 e = E[i];
    const double2 xc = make_double2((double)x0.x, -(double)x0.y);  // conj(x[n])
    const double2 xn = make_double2((double)x0.x, (double)x0.y);
    const double2 ec = cmul(xc, e), en = cmul(xn, e);            // conj(x[n]) E(n), x[n] E(n)
#pragma unroll
    for (int k = 0; k < TT; ++k) {
      if (k < nt) {
        const float2 xl = gload(vx, i + t0 + k);
        const double2 a = make_double2((double)xl.x, (double)xl.y);
        const double2 p0 = cmul(a, ec), p1 = cmul(a, en);
        acc[0][k].x += p0.x;
        acc[0][k].y += p0.y;
        acc[1][k].x += p1.x;
        acc[1][k].y += p1.y;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < TT; ++k) {
    if (k < nt) {
      q[((int64_t)0 * T + t0 + k) * A + r] = acc[0][k];
      q[((int64_t)1 * T + t0 + k) * A + r] = acc[1][k];
    }
  }
}

__device__ __forceinline__ int bitrev(int i, int bits) { return (int)(__brev((unsigned)i) >> (32 - bits)); }

// Row-wise DFT, first stage.  Row `row` of src holds A values; for each
// residue j < P the M = A/P values src[row][P i + j] are transformed by an
// in-place radix-2 FFT in LDS: Y[row][j][k1] = sum_i src[row][P i + j] w_M^{i k1}.
// With P == 1 the result is scaled by `scale` and written straight to the
// output tables (out_mode 1: complex64, 2: complex128).
__global__ __launch_bounds__(256) void grid_fft_kernel(const double2* src, double2* Y, int A, int M, int logM, int P,
                                                        const double2* tw, int T, double scale, int out_mode,
                                                        void* d_R, void* d_Rc) {
  __shared__ double2 buf[FFT_MAX];
  // Block b: rows come in groups of 8; within a group b = 8 j + (row mod 8), so
  // the P sub-transforms of a row, which read interleaved elements of the same
  // lines, are dispatched together and, with workgroups dealt round-robin over
  // the eight XCDs, share one XCD's L2.
  const int grp = blockIdx.x / (8 * P), rem = blockIdx.x % (8 * P);
  const int row = grp * 8 + rem % 8, j = rem / 8, tid = threadIdx.x;
  if (row >= 2 * T) return;
  const double2* s = src + (int64_t)row * A;
  for (int i = tid; i < M; i += 256) buf[bitrev(i, logM)] = s[(int64_t)P * i + j];
  __syncthreads();
  const int tstride = A / M;  // w_M^m = tw[m * A / M]
  constexpr int NBF = FFT_MAX / 512;  // butterflies per thread per stage, at most
  for (int h = 1; h < M; h <<= 1) {
    const int step = tstride * (M / (2 * h));
    // the stage's twiddles first, all loads in flight together (index 0 for
    // butterflies past M/2, whose values are not used)
    double2 w[NBF];
#pragma unroll
    for (int q = 0; q < NBF; ++q) {
      const int b = tid + q * 256;
      w[q] = tw[b < M / 2 ? (int64_t)(b & (h - 1)) * step : 0];
    }
#pragma unroll
    for (int q = 0; q < NBF; ++q) {
      const int b = tid + q * 256;
      if (b < M / 2) {
        const int jj = b & (h - 1);
        const int i0 = ((b - jj) << 1) + jj, i1 = i0 + h;
        const double2 u = buf[i0], t = cmul(w[q], buf[i1]);
        buf[i0] = make_double2(u.x + t.x, u.y + t.y);
        buf[i1] = make_double2(u.x - t.x, u.y - t.y);
      }
    }
    __syncthreads();
  }
  if (P == 1) {
    const int tab = row / T, t = row % T;
    void* base = tab ? d_Rc : d_R;
    if (!base) return;
    for (int k = tid; k < M; k += 256) {
      const double2 v = buf[k];
      const int64_t o = (int64_t)t * A + k;
      if (out_mode == 2)
        reinterpret_cast<double2*>(base)[o] = make_double2(v.x * scale, v.y * scale);
      else
        reinterpret_cast<float2*>(base)[o] = make_float2((float)(v.x * scale), (float)(v.y * scale));
    }
  } else {
    double2* y = Y + ((int64_t)row * P + j) * M;
    for (int k = tid; k < M; k += 256) y[k] = buf[k];
  }
}

// Second stage for A = P M (P <= 8): X[k1 + m M] = sum_{j<P} Y[j][k1] w_A^{j k1} w_P^{j m},
// one thread per (table row, k1) forming all P outputs of k1 from the P
// twiddled inputs, scaled and written to the output tables.
constexpr int COMBINE_MAX = 8;
static_assert(65536 / FFT_MAX <= COMBINE_MAX, "A <= 65536 splits into at most COMBINE_MAX rows");
__global__ void grid_combine_kernel(const double2* Y, int A, int M, int P, const double2* tw, int T, double scale,
                                    int out_mode, void* d_R, void* d_Rc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)2 * T * M) return;
  const int row = (int)(idx / M), k1 = (int)(idx % M);
  const int tab = row / T, t = row % T;
  void* base = tab ? d_Rc : d_R;
  if (!base) return;
  const double2* y = Y + (int64_t)row * P * M;
  double2 v[COMBINE_MAX];
  int e = 0;  // j k1 mod A
#pragma unroll
  for (int j = 0; j < COMBINE_MAX; ++j) {
    if (j < P) {
      v[j] = cmul(tw[e], y[(int64_t)j * M + k1]);
      e += k1;
      e = e >= A ? e - A : e;
    }
  }
  for (int m = 0; m < P; ++m) {
    double2 s = make_double2(0.0, 0.0);
    int f = 0;  // j m M mod A
#pragma unroll
    for (int j = 0; j < COMBINE_MAX; ++j) {
      if (j < P) {
        const double2 u = cmul(tw[f], v[j]);
        s.x += u.x;
        s.y += u.y;
        f += m * M;
        f = f >= A ? f - A : f;
      }
    }
    const int64_t o = (int64_t)t * A + k1 + (int64_t)m * M;
    if (out_mode == 2)
      reinterpret_cast<double2*>(base)[o] = make_double2(s.x * scale, s.y * scale);
    else
      reinterpret_cast<float2*>(base)[o] = make_float2((float)(s.x * scale), (float)(s.y * scale));
  }
}

__global__ void grid_twiddle_kernel(int A, double2* tw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A) return;
  double s, c;
  sincospi(2.0 * (double)i / (double)A, &s, &c);
  tw[i] = make_double2(c, -s);
}

__global__ void grid_zero_kernel(double2* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_double2(0.0, 0.0);
}

__global__ void grid_zero_out_kernel(void* p, int64_t n_bytes4) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_bytes4) reinterpret_cast<uint32_t*>(p)[i] = 0u;
}

__global__ void grid_copy_kernel(VSrc v, int64_t from, int64_t n, float2* dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = gload(v, from + i);
}

inline unsigned nblk(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace grid
}  // namespace cyclo

using namespace cyclo;
using namespace cyclo::grid;

struct cyc_grid {
  int T = 0, A = 0, logA = 0;
  uint32_t flags = 0;
  double alpha0 = 0.0;  // reduced to [-1/2, 1/2]
  int64_t L = 0;        // samples pushed
  int64_t nc = 0;       // products folded (absolute index of pend[cur][0])
  double2* q = nullptr;
  double2* Y = nullptr;
  double2* tw = nullptr;
  double2* E = nullptr;
  float2* pend[2] = {nullptr, nullptr};   // leading input x, from absolute index nc + dx
  float2* pendy[2] = {nullptr, nullptr};  // trailing input y, from nc + dy (two inputs)
  int cur = 0;
  bool two = false;
  int64_t dx = 0, dy = 0, lagabs = 0;
  bool poisoned = false;
  bool zero_q = false;  // q is cleared on the stream of the next push (after a reset)
};

namespace {

void grid_free(cyc_grid* g) {
  if (!g) return;
  (void)hipFree(g->q);
  (void)hipFree(g->Y);
  (void)hipFree(g->tw);
  (void)hipFree(g->E);
  (void)hipFree(g->pend[0]);
  (void)hipFree(g->pend[1]);
  (void)hipFree(g->pendy[0]);
  (void)hipFree(g->pendy[1]);
  delete g;
}

template <typename T>
hipError_t galloc(T** p, size_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T));
}

int grid_fail(cyc_grid* g) {
  g->poisoned = true;
  return CYC_EDEVICE;
}

}  // namespace

extern "C" {

static int grid_create(cyc_grid** out, double alpha0, int32_t n_alpha, int64_t lag_min, int32_t n_lag,
                       uint32_t flags, bool two, void* stream) {
  if (!out || n_lag < 1 || n_lag > 4096 || !std::isfinite(alpha0)) return CYC_EINVAL;
  if (lag_min < -(1 << 20) || lag_min > (1 << 20)) return CYC_EINVAL;
  if (flags & ~CYC_OUT_C128) return CYC_EINVAL;
  if (n_alpha < 2 || n_alpha > 65536 || (n_alpha & (n_alpha - 1)) != 0) return CYC_EUNSUPPORTED;
  cyc_grid* g = new (std::nothrow) cyc_grid();
  if (!g) return CYC_ENOMEM;
  g->T = n_lag;
  g->A = n_alpha;
  while ((1 << g->logA) < n_alpha) ++g->logA;
  g->flags = flags;
  g->alpha0 = alpha0 - std::nearbyint(alpha0);
  g->two = two;
  g->dx = std::max<int64_t>(0, lag_min);
  g->dy = std::max<int64_t>(0, -lag_min);
  g->lagabs = lag_min < 0 ? -lag_min : lag_min;
  const int64_t PC = (int64_t)g->T + g->lagabs;  // pending samples of either input
  const int64_t TA2 = 2 * (int64_t)g->T * g->A;
  if (galloc(&g->q, TA2) != hipSuccess || galloc(&g->tw, g->A) != hipSuccess ||
      galloc(&g->E, MAXP) != hipSuccess || galloc(&g->pend[0], PC) != hipSuccess ||
      galloc(&g->pend[1], PC) != hipSuccess ||
      (two && (galloc(&g->pendy[0], PC) != hipSuccess || galloc(&g->pendy[1], PC) != hipSuccess)) ||
      (g->A > FFT_MAX && galloc(&g->Y, TA2) != hipSuccess)) {
    grid_free(g);
    return CYC_ENOMEM;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(grid_twiddle_kernel, dim3(nblk(g->A)), dim3(256), 0, st, g->A, g->tw);
  hipLaunchKernelGGL(grid_zero_kernel, dim3(nblk(TA2)), dim3(256), 0, st, g->q, TA2);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    grid_free(g);
    return CYC_EDEVICE;
  }
  *out = g;
  return CYC_OK;
}

int cyc_grid_create(cyc_grid** out, double alpha0, int32_t n_alpha, int32_t n_lag, uint32_t flags, void* stream) {
  return grid_create(out, alpha0, n_alpha, 0, n_lag, flags, false, stream);
}

int cyc_grid_create2(cyc_grid** out, double alpha0, int32_t n_alpha, int64_t lag_min, int32_t n_lag,
                     uint32_t flags, void* stream) {
  return grid_create(out, alpha0, n_alpha, lag_min, n_lag, flags, true, stream);
}

}  // extern "C"

namespace {

// One input's virtual array for a push: pending samples from absolute index
// nc + d, then the part of the new block from that index on.
VSrc grid_src(const cyc_grid* g, float2* const* bufs, int64_t d, const float2* blk, int64_t n) {
  const int64_t n_pend = std::max<int64_t>(0, g->L - (g->nc + d));
  const int64_t skip = std::min<int64_t>(n, std::max<int64_t>(0, g->nc + d - g->L));
  VSrc v;
  v.pend = bufs[g->cur];
  v.xin = blk + skip;
  v.n_pend = n_pend;
  v.n_avail = n_pend + (n - skip);
  return v;
}

int grid_push_xy(cyc_grid* g, const float2* x, const float2* y, int64_t n, hipStream_t st) {
  if (g->zero_q) {
    const int64_t TA2 = 2 * (int64_t)g->T * g->A;
    hipLaunchKernelGGL(grid_zero_kernel, dim3(nblk(TA2)), dim3(256), 0, st, g->q, TA2);
    g->zero_q = false;
  }
  const int64_t L_new = g->L + n;
  const int64_t nu_new = std::max<int64_t>(0, L_new - (g->T - 1) - g->lagabs);
  const int64_t np = nu_new - g->nc;  // products that now have all their samples
  const VSrc vx = grid_src(g, g->pend, g->dx, x, n);
  const VSrc vy = g->two ? grid_src(g, g->pendy, g->dy, y, n) : vx;
  // one lag per thread when eight would leave fewer than 1024 workgroups (the
  // loads of the trailing sample and the phase repeat per lag but hit in cache;
  // 2^24 samples, 4096 bins, 128 lags: 5.9 ms per record against 9.0 with eight
  // lags per thread and 6.2 with two)
  const int tt = (int64_t)nblk(g->A, FOLD_NT) * ((g->T + FOLD_TT - 1) / FOLD_TT) < 1024 ? 1 : FOLD_TT;
  const dim3 fgrid(nblk(g->A, FOLD_NT), (unsigned)((g->T + tt - 1) / tt));
  const auto fold = tt == 1 ? grid_fold_kernel<1> : grid_fold_kernel<FOLD_TT>;
  auto shifted = [](VSrc v, int64_t k) {  // the same array from element k on
    if (k < v.n_pend) {
      v.pend += k;
      v.n_pend -= k;
    } else {
      v.xin += k - v.n_pend;
      v.pend = v.xin;
      v.n_pend = 0;
    }
    v.n_avail -= k;
    return v;
  };
  for (int64_t done = 0; done < np;) {
    const int64_t m = std::min<int64_t>(MAXP, np - done);
    const VSrc sx = done > 0 ? shifted(vx, done) : vx;
    const VSrc sy = done > 0 ? shifted(vy, done) : vy;
    hipLaunchKernelGGL(grid_phase_kernel, dim3(nblk(m)), dim3(256), 0, st, g->alpha0, g->nc + done + g->dy, m,
                       g->E);
    // the phase and the fold bin follow y's index: product n goes to bin (n + dy) mod A
    hipLaunchKernelGGL(fold, fgrid, dim3(FOLD_NT), 0, st, sx, sy, g->nc + done + g->dy, m, g->E, g->T,
                       g->A, g->q);
    if (hipGetLastError() != hipSuccess) return grid_fail(g);
    done += m;
  }
  // keep each input's samples from nu_new + d on (fewer than T + |lag_min|)
  const int64_t kx = L_new - (nu_new + g->dx), ky = L_new - (nu_new + g->dy);
  if (kx > 0)
    hipLaunchKernelGGL(grid_copy_kernel, dim3(nblk(kx)), dim3(256), 0, st, vx, np, kx, g->pend[g->cur ^ 1]);
  if (g->two && ky > 0)
    hipLaunchKernelGGL(grid_copy_kernel, dim3(nblk(ky)), dim3(256), 0, st, vy, np, ky, g->pendy[g->cur ^ 1]);
  if (hipGetLastError() != hipSuccess) return grid_fail(g);
  g->cur ^= 1;
  g->L = L_new;
  g->nc = nu_new;
  return CYC_OK;
}

}  // namespace

extern "C" {

int cyc_grid_push(cyc_grid* g, const void* d_x, int64_t n, void* stream) {
  if (!g || n < 0 || (n > 0 && !d_x)) return CYC_EINVAL;
  if (g->poisoned) return CYC_ESTATE;
  if (n == 0) return CYC_OK;
  const float2* x = reinterpret_cast<const float2*>(d_x);
  return grid_push_xy(g, x, x, n, reinterpret_cast<hipStream_t>(stream));
}

int cyc_grid_push2(cyc_grid* g, const void* d_x, const void* d_y, int64_t n, void* stream) {
  if (!g || n < 0 || (n > 0 && (!d_x || !d_y)) || !g->two) return CYC_EINVAL;
  if (g->poisoned) return CYC_ESTATE;
  if (n == 0) return CYC_OK;
  return grid_push_xy(g, reinterpret_cast<const float2*>(d_x), reinterpret_cast<const float2*>(d_y), n,
                      reinterpret_cast<hipStream_t>(stream));
}

int cyc_grid_read(cyc_grid* g, void* d_R, void* d_Rc, int64_t* n_used, void* stream) {
  if (!g) return CYC_EINVAL;
  if (g->poisoned) return CYC_ESTATE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t nu = g->nc;
  if (n_used) *n_used = nu;
  const int out_mode = (g->flags & CYC_OUT_C128) ? 2 : 1;
  const int64_t TA = (int64_t)g->T * g->A;
  if (!d_R && !d_Rc) return CYC_OK;
  if (nu == 0) {
    const int64_t words = TA * (out_mode == 2 ? 4 : 2);
    if (d_R) hipLaunchKernelGGL(grid_zero_out_kernel, dim3(nblk(words)), dim3(256), 0, st, d_R, words);
    if (d_Rc) hipLaunchKernelGGL(grid_zero_out_kernel, dim3(nblk(words)), dim3(256), 0, st, d_Rc, words);
    return hipGetLastError() == hipSuccess ? CYC_OK : grid_fail(g);
  }
  const int M = std::min(g->A, FFT_MAX), P = g->A / M;
  int logM = 0;
  while ((1 << logM) < M) ++logM;
  const double scale = 1.0 / (double)nu;
  hipLaunchKernelGGL(grid_fft_kernel, dim3((unsigned)((2 * g->T + 7) / 8 * 8 * P)), dim3(256), 0, st, g->q, g->Y,
                     g->A, M, logM, P, g->tw, g->T, scale, out_mode, d_R, d_Rc);
  if (P > 1)
    hipLaunchKernelGGL(grid_combine_kernel, dim3(nblk(2 * (int64_t)g->T * M)), dim3(256), 0, st, g->Y, g->A, M, P,
                       g->tw, g->T, scale, out_mode, d_R, d_Rc);
  return hipGetLastError() == hipSuccess ? CYC_OK : grid_fail(g);
}

int cyc_grid_reset(cyc_grid* g) {
  if (!g) return CYC_EINVAL;
  g->zero_q = true;  // the fold bins are cleared by the next push, on its stream
  g->L = 0;
  g->nc = 0;
  g->cur = 0;
  g->poisoned = false;
  return CYC_OK;
}

void cyc_grid_destroy(cyc_grid* g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  grid_free(g);
}

}  // extern "C"
