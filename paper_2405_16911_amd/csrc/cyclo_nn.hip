// Learned cycle-frequency proposal on gfx950: features, network, training,
// labels and selection (cyc_model_* / cyc_select / cyc_peak_labels).
//
// Network (fixed shape): 3 input channels x 1024 bins -> 4 circular conv1d
// layers (64 channels, kernel 7, ReLU) -> dense 64*1024 -> 1024 -> sigmoid.
// Activations are kept channel-major, [C][windows * 1024], so each
// convolution is one matrix product over (windows x positions):
//   forward  U  = W  (Cout x Cin*7) . col (Cin*7 x N)       col = circular im2col
//                                                            (read in place, never stored)
//   backward dW = dU (Cout x N) . col^T,   dcol = W^T . dU,  dX = col2im(dcol)
// and the head is  Z (B x 1024) = H (B x 65536) . Wh^T  with H the flattened
// last activation.  All products run on one MFMA GEMM kernel with FP32 or
// BF16 operands and FP32 accumulation; parameters, gradients and AdamW
// moments are FP32 (the BF16 operands are rounded from the FP32 masters).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "../../include/cyclo.h"
#include "cyclo_internal.h"

namespace cyclo {
namespace nn {

constexpr int CIN = 3, CH = 64, KW = 7, LEN = 1024, NOUT = 1024, NCONV = 4, WIN = 65536, NSEG = 64;
constexpr int LABEL_WIN = 1024;  // largest label window (3 coarse bins of fine bins)
static_assert(NOUT == LEN, "the local layer maps spectral position j to coarse bin j");
static_assert((LEN & (LEN - 1)) == 0, "circular convolution indices wrap with a mask");
constexpr int HDIM = CH * LEN;  // flattened head input

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  bf16x2 v;
  v.x = (__bf16)a;
  v.y = (__bf16)b;
  return __builtin_bit_cast(uint32_t, v);
}

// ----------------------------------------------------------------------------- GEMM
//
// C[M][N] (row-major, ldc) (+)= op(A) . op(B), op(A)[m][k] = TA ? A[k*lda+m] : A[m*lda+k],
// op(B)[k][n] = TB ? B[n*ldb+k] : B[k*ldb+n].  Four waves of 64x64 (2x2 blocks
// of 32x32 MFMA) tile BM x BN = 128 x 128 (WMW = 2) or 64 x 256 (WMW = 1, for
// M <= 64), in 32-deep K steps.  Tiles are staged in LDS k-contiguous: in BF16
// mode as packed pairs, each value rounded to BF16 once while it is staged; in
// FP32 mode as floats.  The LDS tiles are double-buffered and the next step's
// global loads are issued before this step's matrix-core work, one barrier per
// step.  Split K: block z covers k in [z*kchunk, (z+1)*kchunk) and, when part
// is set, writes its partial product to part[z][M][N] for splitk_reduce_kernel.
// With BIM, B holds activations a[ci][ldb] and the GEMM reads their im2col
// matrix col[ci*KW + kk][b*LEN + t] = a[ci][b*LEN + (t + kk - KW/2) mod LEN]
// in place of B (op(B) = col for TB = 0, col^T for TB = 1), so the matrix is
// never written out.
template <int PREC, int TA, int TB, int WMW, int BIM>
__global__ __launch_bounds__(256) void gemm_kernel(const float* __restrict__ A,
                                                   const float* __restrict__ B, float* __restrict__ C,
                                                   int M, int N, int K, int lda, int ldb, int ldc,
                                                   int accumulate, int kchunk, float* __restrict__ part) {
  constexpr int BM = 64 * WMW, BN = 64 * (4 / WMW), BK = 32;
  constexpr int TWD = PREC ? BK / 2 : BK;  // LDS words per tile row: BF16 pairs or floats
  constexpr int LP = TWD + 4;              // row pitch in words, rows 16-byte aligned
  constexpr int NA = BM * TWD / 256, NB = BN * TWD / 256;  // words each thread stages
  __shared__ __attribute__((aligned(16))) uint32_t As[2][BM][LP];
  __shared__ __attribute__((aligned(16))) uint32_t Bs[2][BN][LP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WMW, wn = wave / WMW, h = lane >> 5, l32 = lane & 31;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  const int kbeg = blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);
  // Element (row r, k) of op(X) with bounds check; the load is unconditional
  // (from element 0 when out of range) and the value is masked afterwards.
  auto ld = [](const float* X, int ldx, bool trans, int r, int nr, int k, int kend_) {
    const bool ok = r < nr && k < kend_;
    const float v = X[ok ? (trans ? (int64_t)k * ldx + r : (int64_t)r * ldx + k) : 0];
    return ok ? v : 0.f;
  };
  // word w of tile row r holds k = k0 + 2w, k0 + 2w + 1 (BF16) or k = k0 + w (FP32);
  // thread e stages word (e % TWD) of row (e / TWD), or, when consecutive rows
  // are adjacent in memory (A with TA, B without TB), word (e / rows) of row
  // (e % rows), so that neighbouring threads load neighbouring elements
  // element op(B)[k][r] (r < N), through the im2col map when BIM
  auto ldb_ = [&](int r, int k) {
    const bool ok = r < N && k < kend;
    int64_t addr;
    if (BIM) {
      const int q = TB ? r : k, p = TB ? k : r;  // im2col row and position
      const int ci = q / KW, kk = q - ci * KW, t = p & (LEN - 1);
      addr = (int64_t)ci * ldb + (p - t) + ((t + kk - KW / 2) & (LEN - 1));
    } else {
      addr = TB ? (int64_t)r * ldb + k : (int64_t)k * ldb + r;
    }
    const float v = B[ok ? addr : 0];
    return ok ? v : 0.f;
  };
  uint32_t ra[NA], rb[NB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + i * 256;
      const int r = TA ? e % BM : e / TWD, w = TA ? e / BM : e % TWD;
      if (PREC)
        ra[i] = pack_bf16(ld(A, lda, TA, m0 + r, M, k0 + 2 * w, kend), ld(A, lda, TA, m0 + r, M, k0 + 2 * w + 1, kend));
      else
        ra[i] = __float_as_uint(ld(A, lda, TA, m0 + r, M, k0 + w, kend));
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int e = tid + i * 256;
      const int r = TB ? e / TWD : e % BN, w = TB ? e % TWD : e / BN;
      if (PREC)
        rb[i] = pack_bf16(ldb_(n0 + r, k0 + 2 * w), ldb_(n0 + r, k0 + 2 * w + 1));
      else
        rb[i] = __float_as_uint(ldb_(n0 + r, k0 + w));
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + i * 256;
      As[buf][TA ? e % BM : e / TWD][TA ? e / BM : e % TWD] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int e = tid + i * 256;
      Bs[buf][TB ? e / TWD : e % BN][TB ? e % TWD : e / BN] = rb[i];
    }
  };
  auto compute = [&](int buf) {
    if (PREC == 1) {
#pragma unroll
      for (int kb = 0; kb < BK / 16; ++kb) {
        uint4 af[2], bf[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          af[r] = *reinterpret_cast<const uint4*>(&As[buf][wm * 64 + r * 32 + l32][kb * 8 + 4 * h]);
          bf[r] = *reinterpret_cast<const uint4*>(&Bs[buf][wn * 64 + r * 32 + l32][kb * 8 + 4 * h]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, af[i]), __builtin_bit_cast(bf16x8, bf[j]), acc[i][j], 0, 0, 0);
      }
    } else {
#pragma unroll 4
      for (int k = 0; k < BK; k += 2) {
        float af[2], bf[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          af[r] = __uint_as_float(As[buf][wm * 64 + r * 32 + l32][k + h]);
          bf[r] = __uint_as_float(Bs[buf][wn * 64 + r * 32 + l32][k + h]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
    }
  };

  if (kbeg < kend) {
    fetch(kbeg);
    stash(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
      const bool more = k0 + BK < kend;
      if (more) fetch(k0 + BK);
      compute(buf);
      if (more) stash(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn * 64 + j * 32 + l32;
      if (col >= N) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        if (row >= M) continue;
        if (part) {
          part[((int64_t)blockIdx.z * M + row) * N + col] = acc[i][j][v];
        } else {
          float* c = &C[(int64_t)row * ldc + col];
          *c = accumulate ? *c + acc[i][j][v] : acc[i][j][v];
        }
      }
    }
}

// C[m][n] (+)= sum_z part[z][m][n], z in increasing order
__global__ void splitk_reduce_kernel(const float* __restrict__ part, float* __restrict__ C, int M, int N, int ldc,
                                     int S, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * N) return;
  const int64_t m = i / N, n = i % N;
  float s = 0.f;
  for (int z = 0; z < S; ++z) s += part[(int64_t)z * M * N + i];
  float* c = &C[m * ldc + n];
  *c = accumulate ? *c + s : s;
}

// Launches a GEMM; with fewer output tiles than about two per compute unit the
// K range is split over grid.z (partials in ws, at most ws_cap floats) and
// reduced in a second pass.
hipError_t gemm(int prec, bool ta, bool tb, const float* A, const float* B, float* C, int M, int N, int K,
                int lda, int ldb, int ldc, bool accumulate, hipStream_t st, float* ws = nullptr,
                int64_t ws_cap = 0, bool bim = false) {
  const int wmw = M <= 64 ? 1 : 2;  // 64 x 256 tiles when one 64-row tile covers M
  const int BM = 64 * wmw, BN = 64 * (4 / wmw);
  const int tiles = ((N + BN - 1) / BN) * ((M + BM - 1) / BM);
  int S = 1;
  if (ws && tiles < 512) {
    S = std::min((512 + tiles - 1) / tiles, K / 512);
    while (S > 1 && (int64_t)S * M * N > ws_cap) --S;
    S = std::max(S, 1);
  }
  const int kchunk = S > 1 ? ((K + S - 1) / S + 31) / 32 * 32 : K;
  if (S > 1) S = (K + kchunk - 1) / kchunk;
  float* part = S > 1 ? ws : nullptr;
  const dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, S);
  bool launched = false;
#define GEMM_CASE(P, X, Y, W, I)                                                                         \
  if (!launched && prec == P && ta == (bool)X && tb == (bool)Y && wmw == W && bim == (bool)I) {            \
    hipLaunchKernelGGL((gemm_kernel<P, X, Y, W, I>), grid, dim3(256), 0, st, A, B, C, M, N, K, lda, ldb,    \
                       ldc, accumulate ? 1 : 0, kchunk, part);                                            \
    launched = true;                                                                                      \
  }
#define GEMM_CASES(W)                                                                                     \
  GEMM_CASE(0, 0, 0, W, 0) GEMM_CASE(0, 0, 1, W, 0) GEMM_CASE(0, 1, 0, W, 0) GEMM_CASE(0, 1, 1, W, 0)     \
  GEMM_CASE(1, 0, 0, W, 0) GEMM_CASE(1, 0, 1, W, 0) GEMM_CASE(1, 1, 0, W, 0) GEMM_CASE(1, 1, 1, W, 0)     \
  GEMM_CASE(0, 0, 0, W, 1) GEMM_CASE(0, 0, 1, W, 1) GEMM_CASE(1, 0, 0, W, 1) GEMM_CASE(1, 0, 1, W, 1)
  GEMM_CASES(1) GEMM_CASES(2)
#undef GEMM_CASES
#undef GEMM_CASE
  if (!launched) return hipErrorInvalidValue;
  if (S > 1)
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)(((int64_t)M * N + 255) / 256)), dim3(256), 0, st, ws,
                       C, M, N, ldc, S, accumulate ? 1 : 0);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------- elementwise

inline int nb(int64_t n, int bs = 256) { return (int)((n + bs - 1) / bs); }

// da[ci][b*LEN + s] = sum_k dcol[(ci*KW + k)][b*LEN + (s - k + KW/2) mod LEN]
__global__ void col2im_kernel(const float* dcol, float* da, int cin, int nb_) {
  const int64_t BL = (int64_t)nb_ * LEN;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)cin * BL) return;
  const int ci = (int)(i / BL);
  const int64_t n = i % BL;
  const int64_t b = n / LEN;
  const int s = (int)(n % LEN);
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < KW; ++k) {
    const int t = (s - k + KW / 2 + LEN) % LEN;
    acc += dcol[((int64_t)ci * KW + k) * BL + b * LEN + t];
  }
  da[i] = acc;
}

// u[c][n] += bias[c]; a = max(u, 0)
__global__ void bias_relu_kernel(float* u, const float* bias, float* a, int c, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)c * n) return;
  const float v = u[i] + bias[i / n];
  u[i] = v;
  a[i] = v > 0.f ? v : 0.f;
}

__global__ void relu_bwd_kernel(float* d, const float* u, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(u[i] > 0.f)) d[i] = 0.f;
}

// Row sums in two fixed-order passes: part[r][s] = sum over slice s of the
// columns of X[r][j] (times Y[j] when Y is given), then out[r] = sum_s part[r][s].
constexpr int RSPLIT = 64;

__global__ __launch_bounds__(256) void rowsum_part_kernel(const float* X, const float* Y, float* part,
                                                          int64_t ncol) {
  __shared__ float red[256];
  const int r = blockIdx.x, sl = blockIdx.y;
  const int64_t len = (ncol + RSPLIT - 1) / RSPLIT;
  const int64_t j0 = sl * len, j1 = j0 + len < ncol ? j0 + len : ncol;
  float s = 0.f;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += 256) {
    const float v = X[(int64_t)r * ncol + j];
    s = Y ? fmaf(Y[j], v, s) : s + v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[r * RSPLIT + sl] = red[0];
}

__global__ void rowsum_final_kernel(const float* part, float* out, int rows) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  float s = 0.f;
  for (int k = 0; k < RSPLIT; ++k) s += part[r * RSPLIT + k];
  out[r] = s;
}

// out[o] = sum_b X[b][o]
__global__ void colsum_kernel(const float* X, float* out, int nrow, int ncol) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= ncol) return;
  float s = 0.f;
  for (int b = 0; b < nrow; ++b) s += X[(int64_t)b * ncol + o];
  out[o] = s;
}

// h[b][c*LEN + t] = a[c][b*LEN + t] (dir 0) and the inverse (dir 1)
__global__ void head_layout_kernel(const float* src, float* dst, int nb_, int dir) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)nb_ * HDIM;
  if (i >= tot) return;
  const int64_t b = i / HDIM;
  const int c = (int)((i % HDIM) / LEN), t = (int)(i % LEN);
  const int64_t ia = (int64_t)c * nb_ * LEN + b * LEN + t;  // channel-major index
  if (dir == 0)
    dst[i] = src[ia];
  else
    dst[ia] = src[i];
}

// Local layer (NOUT == LEN): z[b][j] += sum_c Wl[c] * a[c][b*LEN + j], FP32.
__global__ void local_head_kernel(const float* a, const float* Wl, float* z, int nb_) {
  const int64_t BL = (int64_t)nb_ * LEN;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= BL) return;
  float s = 0.f;
  for (int c = 0; c < CH; ++c) s = fmaf(Wl[c], a[(int64_t)c * BL + i], s);
  z[i] += s;
}

// da[c][i] += Wl[c] * dz[i]
__global__ void local_head_dgrad_kernel(float* da, const float* Wl, const float* dz, int64_t BL) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)CH * BL) return;
  da[i] = fmaf(Wl[i / BL], dz[i % BL], da[i]);
}

// z += bias; prob = sigmoid(z); with labels: dz = (prob - y) * scale and
// per-block partial sums of the stable BCE terms.
__global__ void head_out_kernel(float* z, const float* bias, float* prob, const float* y, float* dz,
                                float scale, double* partial, int64_t n) {
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (i < n) {
    const float v = z[i] + bias[i % NOUT];
    z[i] = v;
    const float p = 1.f / (1.f + expf(-v));
    if (prob) prob[i] = p;
    if (y) {
      dz[i] = (p - y[i]) * scale;
      l = (double)fmaxf(v, 0.f) - (double)v * y[i] + log1p(exp(-fabs((double)v)));
    }
  }
  if (!partial) return;
  red[threadIdx.x] = l;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void adamw_kernel(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                             float b2, float eps, float wd, float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / bc1, vh = vi / bc2;
  w[i] = w[i] - lr * (mh / (sqrtf(vh) + eps) + wd * w[i]);
}

// ----------------------------------------------------------------------------- spectra
//
// One workgroup per (window, channel): 64 Hann-windowed 1024-point FFTs
// (radix-2 Stockham in LDS, twiddles exp(-2 pi i m / 1024) from a table made
// in FP64), averaged |X|^2, fftshift, log, standardised over the 1024 bins.
__global__ __launch_bounds__(256) void spectra_kernel(const float2* x, const float2* tw, float* feat,
                                                      int nwin) {
  __shared__ float2 buf[2][LEN];
  __shared__ float P[LEN];
  __shared__ float2 tws[LEN / 2];
  __shared__ double red[256], red2[256];
  const int w = blockIdx.x / 3, ch = blockIdx.x % 3, tid = threadIdx.x;
  for (int i = tid; i < LEN / 2; i += 256) tws[i] = tw[i];
  for (int i = tid; i < LEN; i += 256) P[i] = 0.f;
  __syncthreads();
  const float2* xw = x + (int64_t)w * WIN;
  for (int s = 0; s < NSEG; ++s) {
    for (int i = tid; i < LEN; i += 256) {
      const float2 v = xw[s * LEN + i];
      float2 u;
      if (ch == 0)
        u = v;
      else if (ch == 1)
        u = make_float2(v.x * v.x - v.y * v.y, 2.f * v.x * v.y);
      else
        u = make_float2(v.x * v.x + v.y * v.y, 0.f);
      const float c = i < LEN / 2 ? tws[i].x : -tws[i - LEN / 2].x;  // cos(2 pi i / LEN)
      const float hw = 0.5f - 0.5f * c;
      buf[0][i] = make_float2(u.x * hw, u.y * hw);
    }
    __syncthreads();
    int src = 0;
    for (int ns = 1; ns < LEN; ns <<= 1) {
      for (int j = tid; j < LEN / 2; j += 256) {
        const int k = j & (ns - 1);
        const float2 a0 = buf[src][j], a1 = buf[src][j + LEN / 2];
        const float2 t = tws[k * (LEN / (2 * ns))];
        const float2 b1 = make_float2(a1.x * t.x - a1.y * t.y, a1.x * t.y + a1.y * t.x);
        const int d = (j - k) * 2 + k;
        buf[src ^ 1][d] = make_float2(a0.x + b1.x, a0.y + b1.y);
        buf[src ^ 1][d + ns] = make_float2(a0.x - b1.x, a0.y - b1.y);
      }
      src ^= 1;
      __syncthreads();
    }
    for (int i = tid; i < LEN; i += 256) {
      const float2 v = buf[src][i];
      P[i] += v.x * v.x + v.y * v.y;
    }
    __syncthreads();
  }
  // log of the shifted average, then standardise
  double s1 = 0.0, s2 = 0.0;
  for (int m = tid; m < LEN; m += 256) {
    const double L = log((double)P[(m + LEN / 2) % LEN] / NSEG + 1e-12);
    s1 += L;
    s2 += L * L;
  }
  red[tid] = s1;
  red2[tid] = s2;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (tid < k) {
      red[tid] += red[tid + k];
      red2[tid] += red2[tid + k];
    }
    __syncthreads();
  }
  const double mean = red[0] / LEN;
  const double sd = sqrt(fmax(red2[0] / LEN - mean * mean, 0.0));
  float* out = feat + ((int64_t)ch * nwin + w) * LEN;
  for (int m = tid; m < LEN; m += 256) {
    const double L = log((double)P[(m + LEN / 2) % LEN] / NSEG + 1e-12);
    out[m] = (float)((L - mean) / (sd + 1e-12));
  }
}

__global__ void fft_table_kernel(float2* tw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < LEN / 2) {
    double s, c;
    sincospi(2.0 * (double)i / LEN, &s, &c);
    tw[i] = make_float2((float)c, (float)-s);
  }
}

// ----------------------------------------------------------------------------- labels and selection

// |v| in FP64 as an order-preserving key (non-negative doubles sort like their bits).
__device__ inline unsigned long long mag_key(float2 v) {
  return (unsigned long long)__double_as_longlong(sqrt((double)v.x * v.x + (double)v.y * v.y));
}

// sigma[(tab * T + t) * nc + c] = median of |R_tab[t][a]| over the fine bins a
// of coarse bins c-1, c, c+1 (circular) / sqrt(2 ln 2), the local Rayleigh
// scale of noise-only cells.  A workgroup takes one (table, lag) and a run of
// cb windows: it loads the magnitude keys of coarse bins c0-1 .. c0+cb into
// LDS, one segment of P2 >= per slots per bin (padded with the largest key),
// and sorts every segment at once with a bitonic network.  The key at sorted
// position p of a window is the largest key with at most p keys of the window
// strictly below it; that count is three binary searches, one per sorted
// segment, and an LDS maximum keeps the keys for the two middle positions
// (W-1)/2 and W/2 of W = 3 per.  An even count takes their mean.  A NULL table
// is skipped.
constexpr int SIG_SLOTS = 2048;  // LDS key slots per workgroup: (cb + 2) * P2

__host__ __device__ inline int sig_p2(int per) {
  int p2 = 1;
  while (p2 < per) p2 <<= 1;
  return p2;
}
__host__ __device__ inline int sig_cb(int per, int nc) {
  const int cb = SIG_SLOTS / sig_p2(per) - 2;
  const int lim = nc < SIG_SLOTS / 2 ? nc : SIG_SLOTS / 2;  // windows per workgroup <= the maxima kept
  return cb < 1 ? 1 : (cb > lim ? lim : cb);
}

__global__ __launch_bounds__(256) void local_sigma_kernel(const float2* R, const float2* Rc, int T, int nc,
                                                          int per, double* sigma) {
  __shared__ unsigned long long key[SIG_SLOTS];
  __shared__ unsigned long long mid[SIG_SLOTS / 2][2];
  const int t = blockIdx.y, tab = blockIdx.z, tid = threadIdx.x;
  const float2* base = tab ? Rc : R;
  if (base == nullptr) return;
  const int p2 = sig_p2(per), cb = sig_cb(per, nc);
  const int c0 = blockIdx.x * cb;
  const int nw = min(cb, nc - c0);  // windows of this workgroup
  const int nseg = nw + 2, nkeys = nseg * p2;
  const float2* row = base + (int64_t)t * nc * per;
  for (int i = tid; i < nkeys; i += 256) {
    const int sg = i / p2, j = i % p2;
    int cc = c0 - 1 + sg;
    cc = cc < 0 ? cc + nc : (cc >= nc ? cc - nc : cc);
    key[i] = j < per ? mag_key(row[(int64_t)cc * per + j]) : ~0ull;
  }
  for (int i = tid; i < nw; i += 256) mid[i][0] = mid[i][1] = 0ull;  // keys are >= 0
  __syncthreads();
  // bitonic sort of every segment (ascending)
  for (int k = 2; k <= p2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < nkeys; i += 256) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = ((i % p2) & k) == 0;
          const unsigned long long a = key[i], b = key[l];
          if ((a > b) == up) {
            key[i] = b;
            key[l] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  const int W = 3 * per, lo = (W - 1) / 2, hi = W / 2;
  for (int q = tid; q < nw * W; q += 256) {
    const int w = q / W, e = q % W;
    const unsigned long long k = key[(w + e / per) * p2 + e % per];
    // three independent searches, stepped together; after them keys
    // sgk[d][0 .. pos[d]) are below k
    const unsigned long long* sgk = key + w * p2;
    int pos[3] = {0, p2, 2 * p2};
    for (int st = p2 >> 1; st > 0; st >>= 1) {
#pragma unroll
      for (int d = 0; d < 3; ++d) pos[d] += sgk[pos[d] + st - 1] < k ? st : 0;
    }
    int below = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) below += pos[d] - d * p2 + (sgk[pos[d]] < k ? 1 : 0);
    if (below <= lo) atomicMax(&mid[w][0], k);
    if (below <= hi) atomicMax(&mid[w][1], k);
  }
  __syncthreads();
  for (int w = tid; w < nw; w += 256) {
    const double l = __longlong_as_double((long long)mid[w][0]);
    const double h = __longlong_as_double((long long)mid[w][1]);
    sigma[((int64_t)tab * T + t) * nc + c0 + w] = ((W & 1) ? l : (l + h) / 2.0) / 1.1774100225154747;
  }
}

// label[c] = 1 if some fine bin of coarse bin c exceeds thresh * sigma at some
// lag in either table (the non-conjugate table's zero bin excluded).
__global__ void coarse_label_kernel(const float2* R, const float2* Rc, int T, int nc, int per, int zero_bin,
                                    float thresh, const double* sigma, float* label) {
  const int c = blockIdx.x;
  const int64_t A = (int64_t)nc * per;
  int hit = 0;
  for (int tab = 0; tab < 2; ++tab) {
    if (tab == 0 && c == zero_bin) continue;
    const float2* Rt = tab ? Rc : R;
    if (Rt == nullptr) continue;
    for (int e = threadIdx.x; e < T * per; e += blockDim.x) {
      const int t = e / per, f = e % per;
      const float2 v = Rt[(int64_t)t * A + (int64_t)c * per + f];
      const double m = sqrt((double)v.x * v.x + (double)v.y * v.y);
      if (m > (double)thresh * sigma[((int64_t)tab * T + t) * nc + c]) hit = 1;
    }
  }
  hit = __syncthreads_or(hit);
  if (threadIdx.x == 0) label[c] = hit ? 1.f : 0.f;
}

// Per window: top-k bins of prob (ties -> lower index; NaN bins are never
// chosen), widened by +-width circularly, plus zero_bin; conf = 1 - max prob
// outside the selection, or 0 when any probability is NaN or infinite, or
// (feat given, [3][n][LEN]) any of the window's features is.
__global__ __launch_bounds__(256) void select_kernel(const float* prob, int n, int topk, int width,
                                                     int zero_bin, uint8_t* sel, float* conf,
                                                     const float* feat) {
  __shared__ float p[NOUT];
  __shared__ uint8_t chosen[NOUT], s8[NOUT];
  __shared__ float rv[256];
  __shared__ int ri[256];
  const int w = blockIdx.x, tid = threadIdx.x;
  for (int i = tid; i < NOUT; i += 256) {
    p[i] = prob[(int64_t)w * NOUT + i];
    chosen[i] = 0;
    s8[i] = 0;
  }
  __syncthreads();
  for (int r = 0; r < topk; ++r) {
    float bv = -1.f;
    int bi = NOUT;
    for (int i = tid; i < NOUT; i += 256)
      if (!chosen[i] && (p[i] > bv || (p[i] == bv && i < bi))) {
        bv = p[i];
        bi = i;
      }
    rv[tid] = bv;
    ri[tid] = bi;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
      if (tid < k) {
        const float ov = rv[tid + k];
        const int oi = ri[tid + k];
        if (ov > rv[tid] || (ov == rv[tid] && oi < ri[tid])) {
          rv[tid] = ov;
          ri[tid] = oi;
        }
      }
      __syncthreads();
    }
    if (tid == 0 && ri[0] < NOUT) chosen[ri[0]] = 1;
    __syncthreads();
  }
  for (int i = tid; i < NOUT; i += 256) {
    int s = (i == zero_bin) ? 1 : 0;
    for (int d = -width; d <= width; ++d) s |= chosen[(i + d + NOUT) % NOUT];
    s8[i] = (uint8_t)s;
  }
  __syncthreads();
  float mx = 0.f;
  int bad = 0;
  for (int i = tid; i < NOUT; i += 256) {
    sel[(int64_t)w * NOUT + i] = s8[i];
    if (!s8[i]) mx = fmaxf(mx, p[i]);
    if (!(fabsf(p[i]) <= 3.402823466e38f)) bad = 1;  // NaN or infinite
  }
  if (feat)
    for (int i = tid; i < 3 * NOUT; i += 256)
      if (!(fabsf(feat[((int64_t)(i / NOUT) * n + w) * NOUT + i % NOUT]) <= 3.402823466e38f)) bad = 1;
  rv[tid] = mx;
  bad = __syncthreads_or(bad);
  for (int k = 128; k > 0; k >>= 1) {
    if (tid < k) rv[tid] = fmaxf(rv[tid], rv[tid + k]);
    __syncthreads();
  }
  // a window with a non-finite probability has no confidence: it falls back
  if (tid == 0) conf[w] = bad ? 0.f : 1.f - rv[0];
}

// Per window: the selected coarse bins in ascending order (bins[w][0 .. n)),
// -1 after them, their count, and the fallback flag conf < theta.
__global__ __launch_bounds__(256) void compact_bins_kernel(const uint8_t* sel, const float* conf, float theta,
                                                           int32_t* bins, int32_t* n_bins, uint8_t* fallback) {
  __shared__ int cnt[256];
  const int w = blockIdx.x, tid = threadIdx.x;
  constexpr int PER = NOUT / 256;
  const uint8_t* sw = sel + (int64_t)w * NOUT;
  int c = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) c += sw[tid * PER + k] ? 1 : 0;
  cnt[tid] = c;
  __syncthreads();
  // inclusive scan over the 256 counts (Hillis-Steele, fixed order)
  for (int off = 1; off < 256; off <<= 1) {
    const int v = tid >= off ? cnt[tid - off] : 0;
    __syncthreads();
    cnt[tid] += v;
    __syncthreads();
  }
  const int total = cnt[255];
  int pos = cnt[tid] - c;
  int32_t* bw = bins + (int64_t)w * NOUT;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int b = tid * PER + k;
    if (sw[b]) bw[pos++] = b;
  }
  for (int i = total + tid; i < NOUT; i += 256) bw[i] = -1;
  if (tid == 0) {
    n_bins[w] = total;
    fallback[w] = conf[w] < theta ? 1 : 0;
  }
}

}  // namespace nn
}  // namespace cyclo

using namespace cyclo;
using namespace cyclo::nn;

// ----------------------------------------------------------------------------- model state

struct cyc_model {
  int prec = 0;  // 0: FP32 operands, 1: BF16 operands
  bool local = true;  // the shared local head (CYC_NN_NO_LOCAL turns it off)
  int maxb = 0;
  int64_t np = 0;
  int64_t offW[NCONV], offb[NCONV], offWh = 0, offbh = 0, offWl = 0;
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  int step = 0;
  float* u[NCONV] = {};  // pre-activations [CH][B*LEN]
  float* a[NCONV] = {};  // activations
  float* dcol = nullptr;
  float* hbuf = nullptr;  // [B][HDIM]
  float* z = nullptr;     // [B][NOUT]
  float* dz = nullptr;
  float* da = nullptr;  // [CH][B*LEN]
  float* db2 = nullptr;
  double* partial = nullptr;
  float2* tw = nullptr;
  float* ws = nullptr;  // split-K partial products
  float* rpart = nullptr;  // row-sum partials [CH][RSPLIT]
  int64_t ws_cap = 0;
  float* pfeat = nullptr;    // cyc_propose: features [CIN][B][LEN]
  float* pprob = nullptr;    // cyc_propose: probabilities [B][NOUT]
  uint8_t* psel = nullptr;   // cyc_propose: selection [B][NOUT]
};

namespace {

int64_t model_nparams() {
  int64_t n = 0, cin = CIN;
  for (int i = 0; i < NCONV; ++i) {
    n += (int64_t)CH * cin * KW + CH;
    cin = CH;
  }
  return n + (int64_t)NOUT * HDIM + NOUT + CH;
}

void model_free(cyc_model* m) {
  if (!m) return;
  float* bufs[] = {m->w,  m->g, m->m,  m->v,  m->dcol,  m->hbuf,
                   m->z,  m->dz, m->da, m->db2, m->ws, m->pfeat, m->pprob, m->rpart};
  for (float* p : bufs) (void)hipFree(p);
  for (int i = 0; i < NCONV; ++i) {
    (void)hipFree(m->u[i]);
    (void)hipFree(m->a[i]);
  }
  (void)hipFree(m->partial);
  (void)hipFree(m->tw);
  (void)hipFree(m->psel);
  delete m;
}

template <typename T>
hipError_t dal(T** p, int64_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), (size_t)std::max<int64_t>(count, 1) * sizeof(T));
}

// Forward pass for n windows of features [CIN][n*LEN]; leaves logits in m->z.
hipError_t model_forward(cyc_model* m, const float* feat, int n, hipStream_t st) {
  const int64_t BL = (int64_t)n * LEN;
  const float* in = feat;
  int cin = CIN;
  for (int i = 0; i < NCONV; ++i) {
    // u = W . col(in)
    hipError_t e = gemm(m->prec, false, false, m->w + m->offW[i], in, m->u[i], CH, (int)BL, cin * KW,
                        cin * KW, (int)BL, (int)BL, false, st, m->ws, m->ws_cap, true);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bias_relu_kernel, dim3(nb((int64_t)CH * BL)), dim3(256), 0, st, m->u[i],
                       m->w + m->offb[i], m->a[i], CH, BL);
    in = m->a[i];
    cin = CH;
  }
  hipLaunchKernelGGL(head_layout_kernel, dim3(nb((int64_t)n * HDIM)), dim3(256), 0, st, m->a[NCONV - 1],
                     m->hbuf, n, 0);
  hipError_t e = gemm(m->prec, false, true, m->hbuf, m->w + m->offWh, m->z, n, NOUT, HDIM, HDIM, HDIM, NOUT,
                      false, st, m->ws, m->ws_cap);
  if (e != hipSuccess) return e;
  if (m->local)
    hipLaunchKernelGGL(local_head_kernel, dim3(nb(BL)), dim3(256), 0, st, m->a[NCONV - 1], m->w + m->offWl, m->z,
                       n);
  return hipGetLastError();
}

// Gradients of the mean BCE into m->g; loss partial sums into m->partial.
hipError_t model_backward(cyc_model* m, const float* feat, const float* labels, int n, int* nblk,
                          hipStream_t st) {
  hipError_t e = model_forward(m, feat, n, st);
  if (e != hipSuccess) return e;
  const int64_t nz = (int64_t)n * NOUT;
  *nblk = nb(nz);
  hipLaunchKernelGGL(head_out_kernel, dim3(*nblk), dim3(256), 0, st, m->z, m->w + m->offbh, (float*)nullptr,
                     labels, m->dz, 1.f / (float)nz, m->partial, nz);
  // head
  e = gemm(m->prec, true, false, m->dz, m->hbuf, m->g + m->offWh, NOUT, HDIM, n, NOUT, HDIM, HDIM, false, st,
           m->ws, m->ws_cap);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(colsum_kernel, dim3(nb(NOUT)), dim3(256), 0, st, m->dz, m->g + m->offbh, n, NOUT);
  e = gemm(m->prec, false, false, m->dz, m->w + m->offWh, m->hbuf, n, HDIM, NOUT, NOUT, HDIM, HDIM, false, st,
           m->ws, m->ws_cap);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(head_layout_kernel, dim3(nb((int64_t)n * HDIM)), dim3(256), 0, st, m->hbuf, m->da, n, 1);
  const int64_t BL = (int64_t)n * LEN;
  // dWl[c] = sum_i dz[i] a[c][i]; without the local head its gradient is 0 and
  // it adds nothing to da
  if (m->local) {
    hipLaunchKernelGGL(rowsum_part_kernel, dim3(CH, RSPLIT), dim3(256), 0, st, m->a[NCONV - 1], m->dz, m->rpart, BL);
    hipLaunchKernelGGL(rowsum_final_kernel, dim3(1), dim3(CH), 0, st, m->rpart, m->g + m->offWl, CH);
    hipLaunchKernelGGL(local_head_dgrad_kernel, dim3(nb((int64_t)CH * BL)), dim3(256), 0, st, m->da,
                       m->w + m->offWl, m->dz, BL);
  } else {
    const hipError_t e = cyclo::launch_zero(m->g + m->offWl, sizeof(float) * CH, st);
    if (e != hipSuccess) return e;
  }
  for (int i = NCONV - 1; i >= 0; --i) {
    const int cin = i == 0 ? CIN : CH;
    const float* in = i == 0 ? feat : m->a[i - 1];
    hipLaunchKernelGGL(relu_bwd_kernel, dim3(nb((int64_t)CH * BL)), dim3(256), 0, st, m->da, m->u[i],
                       (int64_t)CH * BL);
    // dW = da . col(in)^T
    e = gemm(m->prec, false, true, m->da, in, m->g + m->offW[i], CH, cin * KW, (int)BL, (int)BL, (int)BL,
             cin * KW, false, st, m->ws, m->ws_cap, true);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rowsum_part_kernel, dim3(CH, RSPLIT), dim3(256), 0, st, m->da, (const float*)nullptr,
                       m->rpart, BL);
    hipLaunchKernelGGL(rowsum_final_kernel, dim3(1), dim3(CH), 0, st, m->rpart, m->g + m->offb[i], CH);
    if (i > 0) {
      e = gemm(m->prec, true, false, m->w + m->offW[i], m->da, m->dcol, cin * KW, (int)BL, CH, cin * KW,
               (int)BL, (int)BL, false, st, m->ws, m->ws_cap);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(col2im_kernel, dim3(nb((int64_t)cin * BL)), dim3(256), 0, st, m->dcol, m->da, cin, n);
    }
  }
  return hipGetLastError();
}

hipError_t loss_from_partials(cyc_model* m, int nblk, int n, double* loss, hipStream_t st) {
  std::vector<double> h(nblk);
  hipError_t e = hipMemcpyAsync(h.data(), m->partial, sizeof(double) * nblk, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  double s = 0.0;
  for (double v : h) s += v;
  *loss = s / ((double)n * NOUT);
  return hipSuccess;
}

}  // namespace

extern "C" {

int64_t cyc_model_num_params(void) { return model_nparams(); }

int cyc_model_create(cyc_model** out, int32_t max_batch, uint32_t flags, void* stream) {
  if (!out || max_batch < 1 || max_batch > 4096) return CYC_EINVAL;
  if (flags & ~(CYC_OP_MASK | CYC_NN_NO_LOCAL)) return CYC_EINVAL;
  const int prec = (int)(flags & CYC_OP_MASK);
  if (prec != 0 && prec != 1) return CYC_EUNSUPPORTED;
  cyc_model* m = new (std::nothrow) cyc_model();
  if (!m) return CYC_ENOMEM;
  m->prec = prec;
  m->local = (flags & CYC_NN_NO_LOCAL) == 0;
  m->maxb = max_batch;
  int64_t o = 0, cin = CIN;
  for (int i = 0; i < NCONV; ++i) {
    m->offW[i] = o;
    o += (int64_t)CH * cin * KW;
    m->offb[i] = o;
    o += CH;
    cin = CH;
  }
  m->offWh = o;
  o += (int64_t)NOUT * HDIM;
  m->offbh = o;
  o += NOUT;
  m->offWl = o;
  o += CH;
  m->np = o;
  const int64_t BL = (int64_t)max_batch * LEN;
  bool ok = dal(&m->w, o) == hipSuccess && dal(&m->g, o) == hipSuccess && dal(&m->m, o) == hipSuccess &&
            dal(&m->v, o) == hipSuccess &&
            dal(&m->dcol, (int64_t)CH * KW * BL) == hipSuccess &&
            dal(&m->hbuf, (int64_t)max_batch * HDIM) == hipSuccess &&
            dal(&m->z, (int64_t)max_batch * NOUT) == hipSuccess &&
            dal(&m->dz, (int64_t)max_batch * NOUT) == hipSuccess && dal(&m->da, (int64_t)CH * BL) == hipSuccess &&
            dal(&m->partial, (int64_t)nb((int64_t)max_batch * NOUT)) == hipSuccess && dal(&m->tw, LEN / 2) == hipSuccess;
  m->ws_cap = (int64_t)1 << 24;
  ok = ok && dal(&m->ws, m->ws_cap) == hipSuccess && dal(&m->pfeat, (int64_t)CIN * BL) == hipSuccess &&
       dal(&m->pprob, (int64_t)max_batch * NOUT) == hipSuccess &&
       dal(&m->psel, (int64_t)max_batch * NOUT) == hipSuccess && dal(&m->rpart, (int64_t)CH * RSPLIT) == hipSuccess;
  for (int i = 0; i < NCONV && ok; ++i)
    ok = dal(&m->u[i], (int64_t)CH * BL) == hipSuccess && dal(&m->a[i], (int64_t)CH * BL) == hipSuccess;
  if (!ok) {
    model_free(m);
    return CYC_ENOMEM;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(fft_table_kernel, dim3(2), dim3(256), 0, st, m->tw);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    model_free(m);
    return CYC_EDEVICE;
  }
  *out = m;
  return CYC_OK;
}

void cyc_model_destroy(cyc_model* m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  model_free(m);
}

int cyc_model_set_params(cyc_model* m, const float* host, void* stream) {
  if (!m || !host) return CYC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(m->w, host, sizeof(float) * m->np, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemsetAsync(m->m, 0, sizeof(float) * m->np, st) != hipSuccess ||
      hipMemsetAsync(m->v, 0, sizeof(float) * m->np, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
    return CYC_EDEVICE;
  m->step = 0;
  return CYC_OK;
}

int cyc_model_get_params(cyc_model* m, float* host, void* stream) {
  if (!m || !host) return CYC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(host, m->w, sizeof(float) * m->np, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return CYC_EDEVICE;
  return CYC_OK;
}

int cyc_model_spectra(cyc_model* m, const void* d_x, int32_t n_windows, float* d_feat, void* stream) {
  if (!m || !d_x || !d_feat || n_windows < 1) return CYC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(spectra_kernel, dim3(n_windows * 3), dim3(256), 0, st, reinterpret_cast<const float2*>(d_x),
                     m->tw, d_feat, n_windows);
  return hipGetLastError() == hipSuccess ? CYC_OK : CYC_EDEVICE;
}

int cyc_model_forward(cyc_model* m, const float* d_feat, int32_t n, float* d_prob, void* stream) {
  if (!m || !d_feat || !d_prob || n < 1 || n > m->maxb) return CYC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (model_forward(m, d_feat, n, st) != hipSuccess) return CYC_EDEVICE;
  const int64_t nz = (int64_t)n * NOUT;
  hipLaunchKernelGGL(head_out_kernel, dim3(nb(nz)), dim3(256), 0, st, m->z, m->w + m->offbh, d_prob,
                     (const float*)nullptr, (float*)nullptr, 0.f, (double*)nullptr, nz);
  return hipGetLastError() == hipSuccess ? CYC_OK : CYC_EDEVICE;
}

int cyc_model_gradients(cyc_model* m, const float* d_feat, const float* d_labels, int32_t n, float* d_grad,
                        double* loss, void* stream) {
  if (!m || !d_feat || !d_labels || n < 1 || n > m->maxb) return CYC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int nblk = 0;
  if (model_backward(m, d_feat, d_labels, n, &nblk, st) != hipSuccess) return CYC_EDEVICE;
  if (d_grad && hipMemcpyAsync(d_grad, m->g, sizeof(float) * m->np, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return CYC_EDEVICE;
  if (loss && loss_from_partials(m, nblk, n, loss, st) != hipSuccess) return CYC_EDEVICE;
  return CYC_OK;
}

int cyc_model_train_step(cyc_model* m, const float* d_feat, const float* d_labels, int32_t n, float lr,
                         float weight_decay, double* loss, void* stream) {
  if (!m || !d_feat || !d_labels || n < 1 || n > m->maxb || !(lr >= 0.f)) return CYC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int nblk = 0;
  if (model_backward(m, d_feat, d_labels, n, &nblk, st) != hipSuccess) return CYC_EDEVICE;
  m->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = 1.f - powf(b1, (float)m->step), bc2 = 1.f - powf(b2, (float)m->step);
  hipLaunchKernelGGL(adamw_kernel, dim3(nb(m->np)), dim3(256), 0, st, m->w, m->g, m->m, m->v, m->np, lr, b1, b2,
                     1e-8f, weight_decay, bc1, bc2);
  if (hipGetLastError() != hipSuccess) return CYC_EDEVICE;
  if (loss && loss_from_partials(m, nblk, n, loss, st) != hipSuccess) return CYC_EDEVICE;
  return CYC_OK;
}

int cyc_select(const float* d_prob, int32_t n, int32_t topk, int32_t width, int32_t zero_bin, uint8_t* d_sel,
               float* d_conf, void* stream) {
  if (!d_prob || !d_sel || !d_conf || n < 1 || topk < 0 || topk > NOUT || width < 0 || width >= NOUT / 2 ||
      zero_bin < -1 || zero_bin >= NOUT)
    return CYC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(select_kernel, dim3(n), dim3(256), 0, st, d_prob, n, topk, width, zero_bin, d_sel, d_conf,
                     (const float*)nullptr);
  return hipGetLastError() == hipSuccess ? CYC_OK : CYC_EDEVICE;
}

int cyc_propose(cyc_model* m, const void* d_x, int32_t n_windows, int32_t topk, int32_t width, int32_t zero_bin,
                float theta, int32_t* d_bins, int32_t* d_n_bins, float* d_conf, uint8_t* d_fallback, void* stream) {
  if (!m || !d_x || !d_bins || !d_n_bins || !d_conf || !d_fallback || n_windows < 1 || n_windows > m->maxb ||
      topk < 0 || topk > NOUT || width < 0 || width >= NOUT / 2 || zero_bin < -1 || zero_bin >= NOUT ||
      !(theta == theta))
    return CYC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int n = n_windows;
  hipLaunchKernelGGL(spectra_kernel, dim3(n * 3), dim3(256), 0, st, reinterpret_cast<const float2*>(d_x), m->tw,
                     m->pfeat, n);
  if (model_forward(m, m->pfeat, n, st) != hipSuccess) return CYC_EDEVICE;
  const int64_t nz = (int64_t)n * NOUT;
  hipLaunchKernelGGL(head_out_kernel, dim3(nb(nz)), dim3(256), 0, st, m->z, m->w + m->offbh, m->pprob,
                     (const float*)nullptr, (float*)nullptr, 0.f, (double*)nullptr, nz);
  // a window with a non-finite feature (a NaN or infinite sample) falls back too:
  // the network's ReLUs would otherwise turn NaN into finite outputs
  hipLaunchKernelGGL(select_kernel, dim3(n), dim3(256), 0, st, m->pprob, n, topk, width, zero_bin, m->psel, d_conf,
                     (const float*)m->pfeat);
  hipLaunchKernelGGL(compact_bins_kernel, dim3(n), dim3(256), 0, st, m->psel, d_conf, theta, d_bins, d_n_bins,
                     d_fallback);
  return hipGetLastError() == hipSuccess ? CYC_OK : CYC_EDEVICE;
}

int cyc_peak_labels(const void* d_R, const void* d_Rc, int32_t n_lag, int32_t n_alpha, int32_t n_coarse,
                    int32_t zero_bin, float thresh, float* d_labels, void* stream) {
  if ((!d_R && !d_Rc) || !d_labels || n_lag < 1 || n_lag > 65535 || n_alpha < 1 || n_coarse < 1 ||
      n_alpha % n_coarse != 0 || 3 * (n_alpha / n_coarse) > LABEL_WIN || zero_bin < -1 || zero_bin >= n_coarse ||
      !(thresh > 0.f))
    return CYC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int per = n_alpha / n_coarse;
  double* sigma = nullptr;
  if (hipMallocAsync(reinterpret_cast<void**>(&sigma), sizeof(double) * 2 * n_lag * (size_t)n_coarse, st) !=
      hipSuccess)
    return CYC_ENOMEM;
  const int sig_cbins = sig_cb(per, n_coarse);
  hipLaunchKernelGGL(local_sigma_kernel, dim3((n_coarse + sig_cbins - 1) / sig_cbins, n_lag, 2), dim3(256), 0, st,
                     reinterpret_cast<const float2*>(d_R), reinterpret_cast<const float2*>(d_Rc), n_lag, n_coarse,
                     per, sigma);
  hipLaunchKernelGGL(coarse_label_kernel, dim3(n_coarse), dim3(256), 0, st, reinterpret_cast<const float2*>(d_R),
                     reinterpret_cast<const float2*>(d_Rc), n_lag, n_coarse, per, zero_bin, thresh, sigma, d_labels);
  const bool ok = hipGetLastError() == hipSuccess;
  (void)hipFreeAsync(sigma, st);
  return ok ? CYC_OK : CYC_EDEVICE;
}

}  // extern "C"
