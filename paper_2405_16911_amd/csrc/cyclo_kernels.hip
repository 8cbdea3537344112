// gfx950 kernels of the streaming cyclic-statistics path.
//
// Contraction.  For one chunk of Kc products starting at sample b the tables
// need, for lags t and cycle frequencies a,
//   S [t][a] = sum_l x[b+l+t] conj(x[b+l]) E(a, b+l)
//   Sc[t][a] = sum_l x[b+l+t]      x[b+l]  E(a, b+l)        (Sec. 4, Eq. (11))
// and E(a, b+l) = E(a, b) * W[l][a] with W[l][a] = exp(-j2pi frac(alpha_a l)).
// The chunk factor E(a, b) is applied later in FP64 (accumulate kernel).  The
// chunk sum is a complex matrix product
//   [S | Sc] = X (T x K) . [Y | Yc] (K x 2A)
// with the Hankel operand X[t][l] = x[b+l+t] (the sample window and its
// lag-shifted copies, staged in LDS without any arithmetic) and the modulated
// operands Y[l][a] = conj(x[b+l]) W[l][a], Yc[l][a] = x[b+l] W[l][a]; the lag
// products x[n+t]x*[n] are formed inside the matrix cores.  Written as one real
// GEMM with the complex parts interleaved along K (k = 2l + c):
//   A'[(t,0)][(l,0)] =  Re x[b+l+t]   A'[(t,0)][(l,1)] = -Im x[b+l+t]
//   A'[(t,1)][(l,0)] =  Im x[b+l+t]   A'[(t,1)][(l,1)] =  Re x[b+l+t]
//   B'[(l,c)][q]     =  component c of Y (q < A) or Yc (q >= A)
// so C'[(t,0)][q] = Re, C'[(t,1)][q] = Im of the table entry, with exactly
// 8 real flops per complex multiply-add and no wasted products.
//
// Twiddles.  W[l][a] = H[a][l / KS] * Lo[a][l % KS] (one complex multiply per
// element) from per-alpha tables made once per state in FP64 (error-free
// alpha*n reduction, FP64 sincospi) and stored in FP32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cyclo_internal.h"

namespace cyclo {

typedef float f32x16 __attribute__((ext_vector_type(16)));

// ----------------------------------------------------------------------------- helpers

__device__ __forceinline__ float2 vload(const VSrc& v, int64_t g) {
  if (g >= v.n_avail) return make_float2(0.f, 0.f);
  const float2* p = g < v.n_pend ? v.pend + g : v.xin + (g - v.n_pend);
  return *p;
}

// Complex product with explicit FMAs, so every kernel that generates operands
// rounds them identically.
__device__ __forceinline__ float2 cmul(float2 p, float2 q) {
  const float t1 = p.y * q.y, t2 = p.y * q.x;
  return make_float2(__fmaf_rn(p.x, q.x, -t1), __fmaf_rn(p.x, q.y, t2));
}

// frac(alpha * n) in [0, 1): error-free product p + e = alpha*n (FMA), then
// (p - floor(p)) + e, wrapped.  |alpha| <= 1/2 and |n| < 2^53.
__device__ __forceinline__ double frac_prod(double alpha, int64_t n) {
  const double nd = (double)n;
  const double p = alpha * nd;
  const double e = __fma_rn(alpha, nd, -p);
  double phi = (p - floor(p)) + e;
  phi -= floor(phi);
  return phi >= 1.0 ? 0.0 : phi;
}

template <int PREC>
struct Op;

template <>
struct Op<PREC_BF16> {
  typedef __bf16 e2 __attribute__((ext_vector_type(2)));
  typedef __bf16 e8 __attribute__((ext_vector_type(8)));
  static __device__ __forceinline__ uint32_t pack(float a, float b) {
    e2 v;
    v.x = (__bf16)a;
    v.y = (__bf16)b;
    return __builtin_bit_cast(uint32_t, v);
  }
  static __device__ __forceinline__ float rnd(float a) { return (float)(__bf16)a; }
  // The two Hankel words of one sample, (re, -im) and (im, re), one packed
  // conversion each (the same rounding as pack).  Written out because the
  // compiler otherwise converts each part once and assembles both words with
  // sign flips and byte permutes, three times the instructions.
  static __device__ __forceinline__ void hankel(float2 v, uint32_t& w0, uint32_t& w1) {
    asm("v_cvt_pk_bf16_f32 %0, %1, -%2" : "=v"(w0) : "v"(v.x), "v"(v.y));
    asm("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(w1) : "v"(v.y), "v"(v.x));
  }
  static __device__ __forceinline__ uint32_t hankel0(float2 v) {
    uint32_t w;
    asm("v_cvt_pk_bf16_f32 %0, %1, -%2" : "=v"(w) : "v"(v.x), "v"(v.y));
    return w;
  }
  static __device__ __forceinline__ uint32_t hankel1(float2 v) {
    uint32_t w;
    asm("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(w) : "v"(v.y), "v"(v.x));
    return w;
  }
  static __device__ __forceinline__ f32x16 mfma(uint4 a, uint4 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(e8, a),
                                                  __builtin_bit_cast(e8, b), c, 0, 0, 0);
  }
};

template <>
struct Op<PREC_F16> {
  typedef _Float16 e2 __attribute__((ext_vector_type(2)));
  typedef _Float16 e8 __attribute__((ext_vector_type(8)));
  // One packed FP32 -> FP16 round-to-nearest conversion, written out: the
  // compiler could otherwise fuse a multiply and the conversion into a mixed
  // FMA that rounds once, and kernels would disagree in the last bit.
  static __device__ __forceinline__ uint32_t pack(float a, float b) {
    uint32_t w;
    asm("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(w) : "v"(a), "v"(b));
    return w;
  }
  static __device__ __forceinline__ float rnd(float a) {
    return (float)__builtin_bit_cast(e2, pack(a, a)).x;
  }
  static __device__ __forceinline__ void hankel(float2 v, uint32_t& w0, uint32_t& w1) {
    asm("v_cvt_pk_f16_f32 %0, %1, -%2" : "=v"(w0) : "v"(v.x), "v"(v.y));
    w1 = pack(v.y, v.x);
  }
  static __device__ __forceinline__ uint32_t hankel0(float2 v) {
    uint32_t w;
    asm("v_cvt_pk_f16_f32 %0, %1, -%2" : "=v"(w) : "v"(v.x), "v"(v.y));
    return w;
  }
  static __device__ __forceinline__ uint32_t hankel1(float2 v) { return pack(v.y, v.x); }
  static __device__ __forceinline__ f32x16 mfma(uint4 a, uint4 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(e8, a),
                                                 __builtin_bit_cast(e8, b), c, 0, 0, 0);
  }
};

// Block index -> (chunk, lag tile, alpha tile).
struct TileId {
  int chunk, tt, at;
};
__device__ __forceinline__ TileId tile_of(const ContractArgs& a) {
  int bid = blockIdx.x;
  TileId r;
  r.at = bid % a.n_at;
  bid /= a.n_at;
  r.tt = bid % a.n_tt;
  r.chunk = bid / a.n_tt;
  return r;
}

// Stores one wave's 32x32 accumulator blocks: rows (t, re/im) interleaved;
// with both tables (TBL = 0) columns q < AW -> table 0 (R) and q >= AW ->
// table 1 (Rc) of the same AW cycle frequencies, with one table (TBL = 1: R,
// 2: Rc) column q is that table at the tile's cycle frequency q (2 AW of them).
template <int WM, int WN, int AW, int TBL>
__device__ __forceinline__ void store_tiles(const ContractArgs& a, const TileId& id, int tau0,
                                            int alpha0, int wm, int wn, int lane,
                                            const f32x16 (&acc)[WM][WN]) {
  const int h = lane >> 5, l32 = lane & 31;
  const int64_t TA = (int64_t)a.T * a.A;
  float2* base = a.part + (int64_t)id.chunk * 2 * TA;
#pragma unroll
  for (int cb = 0; cb < WN; ++cb) {
    const int q = (wn * WN + cb) * 32 + l32;
    const int table = TBL ? TBL - 1 : (q >= AW ? 1 : 0);
    const int alpha = alpha0 + (TBL ? q : q - table * AW);
    if (alpha >= a.A) continue;
    float2* tb = base + table * TA + alpha;
#pragma unroll
    for (int rb = 0; rb < WM; ++rb) {
#pragma unroll
      for (int v = 0; v < 16; v += 2) {
        const int row = 8 * (v >> 2) + 4 * h + (v & 3);
        const int R = (wm * WM + rb) * 32 + row;
        const int tau = tau0 + (R >> 1);
        if (tau < a.T) tb[(int64_t)tau * a.A] = make_float2(acc[rb][cb][v], acc[rb][cb][v + 1]);
      }
    }
  }
}

// ----------------------------------------------------------------------------- sample staging
//
// Each K step of KS products needs the Hankel window Xh[p] = x[s0 + tau0 + p]
// (p < XW) and the modulated-operand samples Xy[j] = x[s0 + j] (j < KS), the
// latter zeroed for products at or beyond the chunk's product count so the
// modulated operands of a partial last step vanish without per-element masks.
// The global loads for step ks+2 (and its twiddle-table entry) are issued
// before the matrix-core work of step ks and written to LDS after it, so their
// latency is hidden.  Loads are bounds-checked, so the steady-state loop can
// stage a window past the last step without branching.  Every lane issues its
// load unconditionally from a valid address (the start of the pending buffer
// when its sample does not exist) and the validity mask is applied when the
// value is written to LDS: a load inside a divergent branch would make the
// compiler wait for it at the branch's join, right after issuing it.
template <int NT, int XW, int KS>
struct Stager {
  static constexpr int N = XW + KS;
  static constexpr int R = (N + NT - 1) / NT;
  float2 r[R];
  bool ok[R];
  float2 hv, hv2;
  // vx: the leading samples (Hankel window), vy: the trailing samples (the
  // modulated operand); the same array for one input.  hp2: the twiddle entry
  // of the thread's second cycle frequency (one-table tiles), else nullptr.
  __device__ __forceinline__ void load(const VSrc& vx, const VSrc& vy, int64_t s0, int tau0, int64_t yend,
                                       const float2* hp, int tid, const float2* hp2 = nullptr) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int idx = tid + i * NT;
      const bool hank = idx < XW;
      const VSrc& v = hank ? vx : vy;
      const int64_t g = hank ? s0 + tau0 + idx : s0 + (idx - XW);
      const bool valid = idx < N && g < v.n_avail && (hank || g < yend);
      const float2* p = valid ? (g < v.n_pend ? v.pend + g : v.xin + (g - v.n_pend)) : v.pend;
      r[i] = *p;
      ok[i] = valid;
    }
    hv = *hp;
    if (hp2) hv2 = *hp2;
  }
  __device__ __forceinline__ void store(float2* Xh, float2* Xy, int tid) const {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int idx = tid + i * NT;
      const float2 val = ok[i] ? r[i] : make_float2(0.f, 0.f);
      if (idx < XW)
        Xh[idx] = val;
      else if (idx < N)
        Xy[idx - XW] = val;
    }
  }
};

// The eight Hankel copies of one K step from the staged window Xh: unit u =
// (sample group u / 4, shift u % 4) holds four consecutive samples in both
// forms (re, -im) at word sh*ZP + 4 grp and (im, re) at CO + sh*ZP + 4 grp.
// When the workgroup has two whole-wave ranges of at least ZU threads, one
// range writes the first form and the other the second (the form is uniform
// per wave), so no unit is done twice; otherwise every thread does whole
// units, and units past ZU repeat earlier ones (identical values to
// identical addresses).
template <typename O, int NT, int ZU, int ZP, int CO>
__device__ __forceinline__ void build_copies(const float2* Xh, uint32_t* Zs, int tid) {
  constexpr int ZUP = (ZU + 63) / 64 * 64;
  if constexpr (2 * ZUP <= NT) {
    const int form = tid >= ZUP;
    const int u = tid - form * ZUP;
    if (u < ZU) {
      const int grp = u >> 2, sh = u & 3;
      uint32_t w[4];
      if (__builtin_amdgcn_readfirstlane(form)) {
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = O::hankel1(Xh[4 * grp + sh + k]);
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = O::hankel0(Xh[4 * grp + sh + k]);
      }
      *reinterpret_cast<uint4*>(&Zs[form * CO + sh * ZP + 4 * grp]) = make_uint4(w[0], w[1], w[2], w[3]);
    }
  } else {
    constexpr int ZR = (ZU + NT - 1) / NT;
#pragma unroll
    for (int i = 0; i < ZR; ++i) {
      const int u = (tid + i * NT) % ZU;
      const int grp = u >> 2, sh = u & 3;
      uint32_t w0[4], w1[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) O::hankel(Xh[4 * grp + sh + k], w0[k], w1[k]);
      *reinterpret_cast<uint4*>(&Zs[sh * ZP + 4 * grp]) = make_uint4(w0[0], w0[1], w0[2], w0[3]);
      *reinterpret_cast<uint4*>(&Zs[CO + sh * ZP + 4 * grp]) = make_uint4(w1[0], w1[1], w1[2], w1[3]);
    }
  }
}

// Modulated operands of one thread: G consecutive samples of one alpha.
// W = H * Lo, Y = conj(x) W, Yc = x W.
template <int G>
__device__ __forceinline__ void modulate(const float2* xs, float2 hv, const float2 (&lo)[G],
                                         float2 (&y)[G], float2 (&yc)[G]) {
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const float2 xv = xs[g];
    const float2 w = cmul(hv, lo[g]);
    const float t1 = xv.y * w.y, t2 = xv.y * w.x;
    y[g] = make_float2(__fmaf_rn(xv.x, w.x, t1), __fmaf_rn(xv.x, w.y, -t2));
    yc[g] = make_float2(__fmaf_rn(xv.x, w.x, -t1), __fmaf_rn(xv.x, w.y, t2));
  }
}


// One table's modulated operand for G consecutive samples of one alpha, with
// the same roundings as modulate: Y = conj(x) W (CONJ = 0, table R) or
// Yc = x W (CONJ = 1, table Rc).
template <int G, int CONJ>
__device__ __forceinline__ void modulate1(const float2* xs, float2 hv, const float2 (&lo)[G], float2 (&y)[G]) {
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const float2 xv = xs[g];
    const float2 w = cmul(hv, lo[g]);
    const float t1 = xv.y * w.y, t2 = xv.y * w.x;
    y[g] = CONJ ? make_float2(__fmaf_rn(xv.x, w.x, -t1), __fmaf_rn(xv.x, w.y, t2))
                : make_float2(__fmaf_rn(xv.x, w.x, t1), __fmaf_rn(xv.x, w.y, -t2));
  }
}

// Common per-workgroup set-up.
struct Tile {
  TileId id;
  int tau0, alpha0, ns, nsteps;
  int64_t cbase, yend;
  __device__ __forceinline__ Tile(const ContractArgs& a, TileId tid_, int tw, int aw, int ks) {
    id = tid_;
    tau0 = id.tt * tw;
    alpha0 = id.at * aw;
    cbase = a.v_off + (int64_t)id.chunk * a.Kc;
    const int64_t mprod = min((int64_t)a.Kc, a.n_prod - (int64_t)id.chunk * a.Kc);
    yend = cbase + mprod;
    nsteps = a.Kc / ks;
    ns = (int)((mprod + ks - 1) / ks);
  }
};

// ----------------------------------------------------------------------------- FP32 contraction
//
// v_mfma_f32_32x32x2f32: one complex sample per instruction (K' = 2 = re, im).
// A lane holds A'[row = lane%32][k = lane/32] and B'[k = lane/32][col = lane%32].
// Hankel value for row (t, cr) and component c: component (cr ^ c) of
// x[s0+l+t], negated for cr = 0, c = 1.
template <int TW, int AW, int WAVES_M, int WAVES_N, int KS, int TBL>
__device__ __forceinline__ void contract_f32_tile(const ContractArgs& a, TileId tid_in) {
  constexpr int NT = 64 * WAVES_M * WAVES_N;
  constexpr int MR = 2 * TW, NC = 2 * AW;
  constexpr int WM = MR / (32 * WAVES_M), WN = NC / (32 * WAVES_N);
  static_assert(WM * 32 * WAVES_M == MR && WN * 32 * WAVES_N == NC, "tile");
  constexpr int G = KS * AW / NT;
  static_assert(G >= 2 && G % 2 == 0 && G * NT == KS * AW && KS % G == 0, "B-gen split");
  constexpr int XW = TW + KS;

  // The matrix-core loop reads the Hankel values straight from the staged
  // window, so it is triple-buffered: the window of step ks+2 is written while
  // slower waves may still read the one of step ks.
  __shared__ __attribute__((aligned(16))) float2 Xh[3][XW];
  __shared__ __attribute__((aligned(16))) float2 Xy[2][KS];
  __shared__ __attribute__((aligned(16))) float2 Bs[2][KS][NC];  // [j][q] = (re, im)

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WAVES_M, wn = wave / WAVES_M;
  const int h = lane >> 5, l32 = lane & 31;
  const Tile tl(a, tid_in, TW, TBL ? 2 * AW : AW, KS);
  const int ns = tl.ns;

  const int ga = tid % AW, gj = (tid / AW) * G;
  const int galpha = tl.alpha0 + ga;
  const bool aval = galpha < a.A;
  float2 lo[G];
#pragma unroll
  for (int g = 0; g < G; ++g)
    lo[g] = aval ? a.Lo[(int64_t)galpha * KS + gj + g] : make_float2(0.f, 0.f);
  const float2* Hcol = a.H + (aval ? galpha : 0);
  auto hptr = [&](int ks) { return Hcol + (int64_t)min(ks, tl.nsteps - 1) * a.hs; };
  // one table: the thread's second cycle frequency (tile column AW + ga)
  const int galpha2 = galpha + AW;
  const bool aval2 = TBL && galpha2 < a.A;
  float2 lo2[TBL ? G : 1];
#pragma unroll
  for (int g = 0; g < (TBL ? G : 1); ++g)
    lo2[g] = aval2 ? a.Lo[(int64_t)galpha2 * KS + gj + g] : make_float2(0.f, 0.f);
  const float2* Hcol2 = a.H + (aval2 ? galpha2 : 0);
  auto hptr2 = [&](int ks) {
    return TBL ? Hcol2 + (int64_t)min(ks, tl.nsteps - 1) * a.hs : (const float2*)nullptr;
  };

  int xoff[WM];
  uint32_t xneg[WM];
#pragma unroll
  for (int rb = 0; rb < WM; ++rb) {
    const int R = (wm * WM + rb) * 32 + l32;
    const int cr = R & 1;
    xoff[rb] = 2 * (R >> 1) + (cr ^ h);
    xneg[rb] = (cr == 0 && h == 1) ? 0x80000000u : 0u;
  }

  auto produce = [&](int buf, float2 hv, float2 hv2) {
    float2 y[G], yc[G];
    if (TBL) {
      float2 lo2g[G];
#pragma unroll
      for (int g = 0; g < G; ++g) lo2g[g] = lo2[TBL ? g : 0];
      modulate1<G, TBL - 1>(&Xy[buf][gj], hv, lo, y);
      modulate1<G, TBL - 1>(&Xy[buf][gj], hv2, lo2g, yc);
    } else {
      modulate<G>(&Xy[buf][gj], hv, lo, y, yc);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      Bs[buf][gj + g][ga] = y[g];
      Bs[buf][gj + g][AW + ga] = yc[g];
    }
  };
  f32x16 acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int k = 0; k < WN; ++k)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][k][v] = 0.f;
  auto mfma_step = [&](int xbuf, int buf) {
    const float* xf = reinterpret_cast<const float*>(&Xh[xbuf][0]);
#pragma unroll 4
    for (int j = 0; j < KS; ++j) {
      float af[WM], bf[WN];
#pragma unroll
      for (int rb = 0; rb < WM; ++rb)
        af[rb] = __uint_as_float(__float_as_uint(xf[2 * j + xoff[rb]]) ^ xneg[rb]);
#pragma unroll
      for (int cb = 0; cb < WN; ++cb)
        bf[cb] = reinterpret_cast<const float*>(&Bs[buf][j][0])[2 * ((wn * WN + cb) * 32 + l32) + h];
#pragma unroll
      for (int rb = 0; rb < WM; ++rb)
#pragma unroll
        for (int cb = 0; cb < WN; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[rb], bf[cb], acc[rb][cb], 0, 0, 0);
    }
  };

  if (ns > 0) {
    Stager<NT, XW, KS> stg;
    stg.load(a.v, a.vy, tl.cbase, tl.tau0, tl.yend, hptr(0), tid, hptr2(0));
    stg.store(&Xh[0][0], &Xy[0][0], tid);
    const float2 h0 = stg.hv, h02 = stg.hv2;
    stg.load(a.v, a.vy, tl.cbase + KS, tl.tau0, tl.yend, hptr(1), tid, hptr2(1));
    stg.store(&Xh[1][0], &Xy[1][0], tid);
    float2 hnext = stg.hv, hnext2 = stg.hv2;
    __syncthreads();
    produce(0, h0, h02);
    __syncthreads();
    int xb = 0;  // = ks % 3
    for (int ks = 0; ks + 1 < ns; ++ks) {
      const int buf = ks & 1;
      const int xb2 = xb == 0 ? 2 : xb - 1;  // (ks + 2) % 3
      stg.load(a.v, a.vy, tl.cbase + (int64_t)(ks + 2) * KS, tl.tau0, tl.yend, hptr(ks + 2), tid,
               hptr2(ks + 2));
      __builtin_amdgcn_s_setprio(1);  // as in the 16-bit kernel
      mfma_step(xb, buf);
      __builtin_amdgcn_s_setprio(0);
      produce(buf ^ 1, hnext, hnext2);
      stg.store(&Xh[xb2][0], &Xy[buf][0], tid);
      hnext = stg.hv;
      hnext2 = stg.hv2;
      xb = xb == 2 ? 0 : xb + 1;
      __syncthreads();
    }
    mfma_step(xb, (ns - 1) & 1);
  }
  store_tiles<WM, WN, AW, TBL>(a, tl.id, tl.tau0, tl.alpha0, wm, wn, lane, acc);
}

// ----------------------------------------------------------------------------- BF16/FP16 contraction
//
// v_mfma_f32_32x32x16_{bf16,f16}: a lane holds A'[row = lane%32][8*(lane/32) + s]
// and B'[8*(lane/32) + s][col = lane%32], s = 0..7, i.e. four consecutive complex
// samples (re, im interleaved) starting at sample 4*(lane/32) of the 8-sample
// K block.  The Hankel operand is kept as eight copies (cr, sh) holding the
// pairs (re, -im) (cr = 0) or (im, re) (cr = 1) of the window shifted by
// sh = 0..3 samples, so every 16-byte fragment read is aligned for any lag.
// Copy (cr, sh) starts at word cr*CO + sh*ZP (ZP and CO below).
template <int PREC, int SPLIT, int TW, int AW, int WAVES_M, int WAVES_N, int KS, int SCHED, int TBL>
__device__ __forceinline__ void contract_16_tile(const ContractArgs& a, TileId tid_in) {
  using O = Op<PREC>;
  constexpr int NT = 64 * WAVES_M * WAVES_N;
  constexpr int MR = 2 * TW, NC = 2 * AW;
  constexpr int WM = MR / (32 * WAVES_M), WN = NC / (32 * WAVES_N);
  static_assert(WM * 32 * WAVES_M == MR && WN * 32 * WAVES_N == NC, "tile");
  static_assert(KS % 8 == 0 && TW % 16 == 0, "shape");
  constexpr int G = KS * AW / NT;
  static_assert(G >= 4 && G * NT == KS * AW && KS % G == 0 && G % 4 == 0, "B-gen split");
  constexpr int ZW = KS + TW;                    // entries per shifted copy (multiple of 4)
  // Copy pitch ZP >= ZW with ZP = 8 (mod 64) words and the cr = 1 copies at
  // CO = 4 ZP.  (A probe of the fragment reads alone found ZP = 32, CO = 16
  // (mod 64) free of the 2-way bank conflicts this layout has, but the kernels
  // ran 0-4% slower with it: its Hankel-copy writes conflict instead.)
  constexpr int ZP = ((ZW + 55) / 64) * 64 + 8;
  constexpr int CO = 4 * ZP;
  constexpr int ZS = CO + 4 * ZP;                // words per buffer
  static_assert(ZP >= ZW && ZP % 64 == 8 && CO % 64 == 32, "Hankel copy layout");
  constexpr int XW = ZW + 4;                     // staged Hankel samples (ZW + 3 are read)
  constexpr int BP = KS + 4;                     // B row pitch (uint32), rows 16-byte aligned
  constexpr int NB = SPLIT ? 2 : 1;
  constexpr int ZU = ZW;                         // staging units: 4 entries x 1 shift x both cr

  __shared__ __attribute__((aligned(16))) uint32_t Zs[2][ZS];
  __shared__ __attribute__((aligned(16))) uint32_t Bs[2][NB][NC][BP];
  __shared__ __attribute__((aligned(16))) float2 Xh[2][XW];
  __shared__ __attribute__((aligned(16))) float2 Xy[2][KS];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WAVES_M, wn = wave / WAVES_M;
  const int h = lane >> 5, l32 = lane & 31;
  const Tile tl(a, tid_in, TW, TBL ? 2 * AW : AW, KS);
  const int ns = tl.ns;

  const int ga = tid % AW, gj = (tid / AW) * G;
  const int galpha = tl.alpha0 + ga;
  const bool aval = galpha < a.A;
  float2 lo[G];
#pragma unroll
  for (int g = 0; g < G; ++g) lo[g] = aval ? a.Lo[(int64_t)galpha * KS + gj + g] : make_float2(0.f, 0.f);
  const float2* Hcol = a.H + (aval ? galpha : 0);
  auto hptr = [&](int ks) { return Hcol + (int64_t)min(ks, tl.nsteps - 1) * a.hs; };
  // one table: the thread's second cycle frequency (tile column AW + ga)
  const int galpha2 = galpha + AW;
  const bool aval2 = TBL && galpha2 < a.A;
  float2 lo2[TBL ? G : 1];
#pragma unroll
  for (int g = 0; g < (TBL ? G : 1); ++g)
    lo2[g] = aval2 ? a.Lo[(int64_t)galpha2 * KS + gj + g] : make_float2(0.f, 0.f);
  const float2* Hcol2 = a.H + (aval2 ? galpha2 : 0);
  auto hptr2 = [&](int ks) {
    return TBL ? Hcol2 + (int64_t)min(ks, tl.nsteps - 1) * a.hs : (const float2*)nullptr;
  };

  // Word offset of this lane's Hankel fragment for the wave's first row block
  // (row R = 2 lag + cr, four samples from lag + 4h, in copy (cr, lag + 4h mod 4)).
  int zoff0;
  {
    const int R = wm * WM * 32 + l32;
    const int p0 = (R >> 1) + 4 * h;
    const int sh = p0 & 3;
    zoff0 = (R & 1) * CO + sh * ZP + (p0 - sh);
  }

  auto produce = [&](int buf, float2 hv, float2 hv2) {
    build_copies<O, NT, ZU, ZP, CO>(&Xh[buf][0], &Zs[buf][0], tid);
    // modulated operands
    uint32_t py[NB][G], pyc[NB][G];
    {
      float2 y[G], yc[G];
      if (TBL) {
        float2 lo2g[G];
#pragma unroll
        for (int g = 0; g < G; ++g) lo2g[g] = lo2[TBL ? g : 0];
        modulate1<G, TBL - 1>(&Xy[buf][gj], hv, lo, y);
        modulate1<G, TBL - 1>(&Xy[buf][gj], hv2, lo2g, yc);
      } else {
        modulate<G>(&Xy[buf][gj], hv, lo, y, yc);
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        py[0][g] = O::pack(y[g].x, y[g].y);
        pyc[0][g] = O::pack(yc[g].x, yc[g].y);
        if (SPLIT) {
          py[NB - 1][g] = O::pack(y[g].x - O::rnd(y[g].x), y[g].y - O::rnd(y[g].y));
          pyc[NB - 1][g] = O::pack(yc[g].x - O::rnd(yc[g].x), yc[g].y - O::rnd(yc[g].y));
        }
      }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int g = 0; g < G; g += 4) {
        *reinterpret_cast<uint4*>(&Bs[buf][b][ga][gj + g]) =
            make_uint4(py[b][g], py[b][g + 1], py[b][g + 2], py[b][g + 3]);
        *reinterpret_cast<uint4*>(&Bs[buf][b][AW + ga][gj + g]) =
            make_uint4(pyc[b][g], pyc[b][g + 1], pyc[b][g + 2], pyc[b][g + 3]);
      }
  };

  f32x16 acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int k = 0; k < WN; ++k)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][k][v] = 0.f;
  // Hankel fragments: row block rb at K block kb reads word zoff0 + 16 rb + 8 kb
  // (the block's lags are 16 further on, and 16 = 0 mod 4 keeps the copy), so
  // block rb + 1 at kb holds the same values as block rb at kb + 2.  Each
  // distinct fragment of a step is read once: 2 (WM - 1) + KS / 8 of them
  // instead of WM * KS / 8.  The next step's window starts KS samples on, so
  // its first NCF fragments are this step's last NCF (the staged samples
  // depend only on their absolute index): they stay in registers, and a step
  // reads only its last KS / 8 fragments from LDS.
  constexpr int NAF = 2 * (WM - 1) + KS / 8;
  constexpr int NCF = 2 * (WM - 1);
  uint4 afc[NCF > 0 ? NCF : 1];
  auto load_carry = [&](int buf) {
    const uint32_t* zb = &Zs[buf][0] + zoff0;
#pragma unroll
    for (int o = 0; o < NCF; ++o) afc[o] = *reinterpret_cast<const uint4*>(zb + 8 * o);
  };
  auto mfma_step = [&](int buf) {
    const uint32_t* zb = &Zs[buf][0] + zoff0;
    uint4 af[NAF];
#pragma unroll
    for (int o = 0; o < NCF; ++o) af[o] = afc[o];
#pragma unroll
    for (int o = NCF; o < NAF; ++o) af[o] = *reinterpret_cast<const uint4*>(zb + 8 * o);
#pragma unroll
    for (int o = 0; o < NCF; ++o) afc[o] = af[KS / 8 + o];
#pragma unroll
    for (int kb = 0; kb < KS / 8; ++kb) {
      const int j0 = kb * 8;
      uint4 bf[NB][WN];
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int cb = 0; cb < WN; ++cb)
          bf[b][cb] = *reinterpret_cast<const uint4*>(
              &Bs[buf][b][(wn * WN + cb) * 32 + l32][j0 + 4 * h]);
#pragma unroll
      for (int rb = 0; rb < WM; ++rb)
#pragma unroll
        for (int cb = 0; cb < WN; ++cb) {
          acc[rb][cb] = O::mfma(af[2 * rb + kb], bf[0][cb], acc[rb][cb]);
          if (SPLIT) acc[rb][cb] = O::mfma(af[2 * rb + kb], bf[NB - 1][cb], acc[rb][cb]);
        }
    }
  };

  // A step's twiddle entries wait in LDS between their load and their use,
  // in the padding words of the B rows (the matrix-core reads stop at word
  // KS): row ga for the thread's cycle frequency, row AW + ga for the second
  // one of a one-table tile.  One thread per cycle frequency writes them.
  auto put_h = [&](int buf, const Stager<NT, XW, KS>& st) {
    if (gj == 0) {
      *reinterpret_cast<float2*>(&Bs[buf][0][ga][KS]) = st.hv;
      if (TBL) *reinterpret_cast<float2*>(&Bs[buf][0][AW + ga][KS]) = st.hv2;
    }
  };
  auto get_h = [&](int buf, int row0) { return *reinterpret_cast<const float2*>(&Bs[buf][0][row0 + ga][KS]); };
  // Sample loads run two K steps ahead: the registers of two stagers
  // alternate, so a load has a whole step (its matrix-core work and operand
  // generation) more to land than it would with one stager, which a short
  // step (64 lags) does not cover at load latencies under full load.
  if (ns > 0) {
    Stager<NT, XW, KS> sa, sb;
    sa.load(a.v, a.vy, tl.cbase, tl.tau0, tl.yend, hptr(0), tid, hptr2(0));
    sa.store(&Xh[0][0], &Xy[0][0], tid);
    const float2 h0 = sa.hv, h02 = sa.hv2;
    sb.load(a.v, a.vy, tl.cbase + KS, tl.tau0, tl.yend, hptr(1), tid, hptr2(1));
    sb.store(&Xh[1][0], &Xy[1][0], tid);
    put_h(1, sb);
    sa.load(a.v, a.vy, tl.cbase + 2 * KS, tl.tau0, tl.yend, hptr(2), tid, hptr2(2));
    __syncthreads();
    produce(0, h0, h02);
    __syncthreads();
    load_carry(0);
    // Step ks: cur holds the loads of step ks + 2, which go to LDS at the end
    // of the step (the thread's twiddle entry too, to its own slot), and nxt
    // takes those of step ks + 3.  No loaded register is carried past the
    // two-step unrolled loop body, so none needs a copy, and a wait for the
    // load, at the back edge.
    auto body = [&](int ks, Stager<NT, XW, KS>& cur, Stager<NT, XW, KS>& nxt) {
      const int buf = ks & 1;
      nxt.load(a.v, a.vy, tl.cbase + (int64_t)(ks + 3) * KS, tl.tau0, tl.yend, hptr(ks + 3), tid,
               hptr2(ks + 3));
      // The wave issuing matrix-core work runs at raised priority; the other
      // resident wave's operand generation fills the issue slots it leaves.
      __builtin_amdgcn_s_setprio(1);
      mfma_step(buf);
      __builtin_amdgcn_s_setprio(0);
      produce(buf ^ 1, get_h(buf ^ 1, 0), get_h(buf ^ 1, TBL ? AW : 0));
      cur.store(&Xh[buf][0], &Xy[buf][0], tid);
      put_h(buf, cur);
      if (SCHED) {
        // Interleave the next step's operand generation with this step's
        // matrix-core instructions so one wave overlaps both.
        // SCHED = 1: four VALU instructions per MFMA, else SCHED of them
        constexpr int NMF = WM * WN * (KS / 8) * NB;
        constexpr int NV = SCHED == 1 ? 4 : SCHED;
#pragma unroll
        for (int i = 0; i < NMF; ++i) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
          __builtin_amdgcn_sched_group_barrier(0x002, NV, 0);  // VALU
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS read
        }
      }
      __syncthreads();
    };
    int ks = 0;
    for (; ks + 2 < ns; ks += 2) {
      body(ks, sa, sb);
      body(ks + 1, sb, sa);
    }
    if (ks + 1 < ns) body(ks, sa, sb);
    mfma_step((ns - 1) & 1);
  }
  store_tiles<WM, WN, AW, TBL>(a, tl.id, tl.tau0, tl.alpha0, wm, wn, lane, acc);
}

// ----------------------------------------------------------------------------- kernels
//
// One workgroup per (chunk, lag tile, alpha tile) of one stream state, and a
// persistent form for a batch of states: a fixed grid whose workgroups take
// work items (job, lag tile, alpha tile) from an atomic counter until the
// list is exhausted.  Every workgroup reaches the exit test each round, so the
// grid drains whatever the number of items.
template <int TW, int AW, int WAVES_M, int WAVES_N, int KS, int TBL>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N, 2) void contract_f32(ContractArgs a) {
  contract_f32_tile<TW, AW, WAVES_M, WAVES_N, KS, TBL>(a, tile_of(a));
}

template <int PREC, int SPLIT, int TW, int AW, int WAVES_M, int WAVES_N, int KS, int SCHED, int TBL>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N, 2) void contract_16(ContractArgs a) {
  contract_16_tile<PREC, SPLIT, TW, AW, WAVES_M, WAVES_N, KS, SCHED, TBL>(a, tile_of(a));
}

// Takes the next work item; all threads of the workgroup see the same value.
__device__ __forceinline__ int next_item(int* counter) {
  __shared__ int item;
  __syncthreads();  // every thread has read the previous item
  if (threadIdx.x == 0) item = atomicAdd(counter, 1);
  __syncthreads();
  return item;
}

__device__ __forceinline__ ContractArgs job_args(const BatchArgs& b, const BJob& j) {
  ContractArgs a;
  a.v = j.v;
  a.vy = j.v;
  a.v_off = j.v_off;
  a.n_prod = j.n_prod;
  a.T = b.T;
  a.A = j.A;
  a.Kc = b.Kc;
  a.n_tt = 1;
  a.n_at = 1;
  a.n_chunks = 1;
  a.H = j.H;
  a.hs = b.hs;
  a.Lo = j.Lo;
  a.part = j.part;
  return a;
}

template <int TW, int AW, int WAVES_M, int WAVES_N, int KS>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N, 2) void contract_f32_batch(BatchArgs b) {
  for (;;) {
    const int it = next_item(b.counter);
    if (it >= *b.n_items) break;
    const BItem bi = b.items[it];
    const BJob j = b.jobs[bi.job];
    TileId id;
    id.chunk = 0;
    id.tt = bi.tt;
    id.at = bi.at;
    contract_f32_tile<TW, AW, WAVES_M, WAVES_N, KS, 0>(job_args(b, j), id);
  }
}

template <int PREC, int SPLIT, int TW, int AW, int WAVES_M, int WAVES_N, int KS, int SCHED>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N, 2) void contract_16_batch(BatchArgs b) {
  for (;;) {
    const int it = next_item(b.counter);
    if (it >= *b.n_items) break;
    const BItem bi = b.items[it];
    const BJob j = b.jobs[bi.job];
    TileId id;
    id.chunk = 0;
    id.tt = bi.tt;
    id.at = bi.at;
    contract_16_tile<PREC, SPLIT, TW, AW, WAVES_M, WAVES_N, KS, SCHED, 0>(job_args(b, j), id);
  }
}

// ----------------------------------------------------------------------------- register-B contraction
//
// BF16/FP16 variant for large lag tiles.  One wave per workgroup owns every
// row of the tile (RB blocks of 32 rows = 16 lags each) and NA blocks of 32
// cycle frequencies.  The modulated operands are generated directly in the
// registers of the matrix-core B fragment (lane = alpha, four consecutive
// samples per lane half), so they never pass through LDS; LDS holds only the
// FP32 sample window and the eight shifted Hankel copies, double-buffered.
// Accumulators: RB x 2NA blocks (Y blocks first, then Yc blocks).
template <int PREC, int SPLIT, int RB, int NA, int KS>
__global__ __launch_bounds__(64, 1) void contract_rg(ContractArgs a) {
  const TileId tid_in = tile_of(a);
  using O = Op<PREC>;
  constexpr int NT = 64;
  constexpr int TW = 16 * RB, AW = 32 * NA;
  static_assert(KS % 8 == 0, "shape");
  constexpr int NKB = KS / 8;                    // 8-sample K blocks per step
  constexpr int ZW = KS + TW;
  constexpr int ZP = ((ZW + 55) / 64) * 64 + 8;  // layout of contract_16_tile
  constexpr int CO = 4 * ZP;
  constexpr int ZS = CO + 4 * ZP;
  constexpr int XW = ZW + 4;
  constexpr int ZU = ZW;
  constexpr int ZR = (ZU + NT - 1) / NT;
  constexpr int NB = SPLIT ? 2 : 1;

  __shared__ __attribute__((aligned(16))) uint32_t Zs[2][ZS];
  __shared__ __attribute__((aligned(16))) float2 Xh[3][XW];
  __shared__ __attribute__((aligned(16))) float2 Xy[3][KS];

  const int tid = threadIdx.x, lane = tid;
  const int h = lane >> 5, l32 = lane & 31;
  const Tile tl(a, tid_in, TW, AW, KS);
  const int ns = tl.ns;

  // lane's cycle frequencies and the chunk-relative twiddles of the samples it
  // generates: j = 8 kb + 4 h + g within a step
  float2 lo[NA][NKB][4];
  const float2* Hrow[NA];
#pragma unroll
  for (int nb = 0; nb < NA; ++nb) {
    const int al = tl.alpha0 + nb * 32 + l32;
    const bool ok = al < a.A;
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
      for (int g = 0; g < 4; ++g)
        lo[nb][kb][g] = ok ? a.Lo[(int64_t)al * KS + 8 * kb + 4 * h + g] : make_float2(0.f, 0.f);
    Hrow[nb] = a.H + (ok ? al : 0);
  }
  auto hidx = [&](int ks) { return (int64_t)min(ks, tl.nsteps - 1) * a.hs; };

  int zoff[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int R = rb * 32 + l32;
    const int p0 = (R >> 1) + 4 * h;
    const int sh = p0 & 3;
    zoff[rb] = (R & 1) * CO + sh * ZP + (p0 - sh);
  }

  auto build_hankel = [&](int xbuf, int buf) {
#pragma unroll
    for (int i = 0; i < ZR; ++i) {
      const int u = (tid + i * NT) % ZU;
      const int grp = u >> 2, sh = u & 3;
      uint32_t w0[4], w1[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        O::hankel(Xh[xbuf][4 * grp + sh + k], w0[k], w1[k]);
      }
      *reinterpret_cast<uint4*>(&Zs[buf][sh * ZP + 4 * grp]) = make_uint4(w0[0], w0[1], w0[2], w0[3]);
      *reinterpret_cast<uint4*>(&Zs[buf][CO + sh * ZP + 4 * grp]) =
          make_uint4(w1[0], w1[1], w1[2], w1[3]);
    }
  };

  f32x16 acc[RB][2 * NA];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int k = 0; k < 2 * NA; ++k)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][k][v] = 0.f;

  // Operands of one 8-sample K block: Hankel fragments from LDS, modulated
  // fragments generated in registers from samples already held in registers.
  struct Frag {
    uint4 a[RB];
    uint4 y[NB][NA], yc[NB][NA];
  };
  typedef float2 StepX[NKB][4];  // this lane's samples of one step: j = 8 kb + 4 h + g
  auto load_x = [&](int xbuf, StepX& xs) {
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
      const float4 xa = *reinterpret_cast<const float4*>(&Xy[xbuf][8 * kb + 4 * h]);
      const float4 xb = *reinterpret_cast<const float4*>(&Xy[xbuf][8 * kb + 4 * h + 2]);
      xs[kb][0] = make_float2(xa.x, xa.y);
      xs[kb][1] = make_float2(xa.z, xa.w);
      xs[kb][2] = make_float2(xb.x, xb.y);
      xs[kb][3] = make_float2(xb.z, xb.w);
    }
  };
  auto fetch = [&](int zbuf, int kb, const StepX& xs, const float2 (&hv)[NA], Frag& f) {
    const uint32_t* zb = &Zs[zbuf][0];
    const int j0 = kb * 8;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) f.a[rb] = *reinterpret_cast<const uint4*>(zb + zoff[rb] + j0);
#pragma unroll
    for (int nb = 0; nb < NA; ++nb) {
      uint32_t py[NB][4], pyc[NB][4];
      {
        float2 y[4], yc[4];
        modulate<4>(xs[kb], hv[nb], lo[nb][kb], y, yc);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          py[0][g] = O::pack(y[g].x, y[g].y);
          pyc[0][g] = O::pack(yc[g].x, yc[g].y);
          if (SPLIT) {
            py[NB - 1][g] = O::pack(y[g].x - O::rnd(y[g].x), y[g].y - O::rnd(y[g].y));
            pyc[NB - 1][g] = O::pack(yc[g].x - O::rnd(yc[g].x), yc[g].y - O::rnd(yc[g].y));
          }
        }
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        f.y[b][nb] = make_uint4(py[b][0], py[b][1], py[b][2], py[b][3]);
        f.yc[b][nb] = make_uint4(pyc[b][0], pyc[b][1], pyc[b][2], pyc[b][3]);
      }
    }
  };
  auto mma = [&](const Frag& f) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int nb = 0; nb < NA; ++nb)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          acc[rb][nb] = O::mfma(f.a[rb], f.y[b][nb], acc[rb][nb]);
          acc[rb][NA + nb] = O::mfma(f.a[rb], f.yc[b][nb], acc[rb][NA + nb]);
        }
  };

  // Software pipeline.  One wave per workgroup: its LDS operations execute in
  // program order, so no barriers are needed, and a buffer is rewritten only
  // after every read of it has been issued.  Sample windows are
  // triple-buffered (Xh/Xy[ks % 3]) and their global loads land a full step
  // before they are written to LDS; Hankel copies are double-buffered
  // (Zs[ks & 1]) and built one step ahead; the step's samples for the
  // modulated operands are read into registers one step ahead.
  if (ns > 0) {
    Stager<NT, XW, KS> stg;
    float2 hc[NA], hn[NA], hnn[NA];
    stg.load(a.v, a.vy, tl.cbase, tl.tau0, tl.yend, Hrow[0] + hidx(0), tid);
    stg.store(&Xh[0][0], &Xy[0][0], tid);
    stg.load(a.v, a.vy, tl.cbase + KS, tl.tau0, tl.yend, Hrow[0] + hidx(1), tid);
    stg.store(&Xh[1][0], &Xy[1][0], tid);
    stg.load(a.v, a.vy, tl.cbase + 2 * KS, tl.tau0, tl.yend, Hrow[0] + hidx(2), tid);
#pragma unroll
    for (int nb = 0; nb < NA; ++nb) {
      hc[nb] = Hrow[nb][hidx(0)];
      hn[nb] = Hrow[nb][hidx(1)];
      hnn[nb] = Hrow[nb][hidx(2)];
    }
    build_hankel(0, 0);
    StepX xc, xn;
    load_x(0, xc);
    Frag cur;
    fetch(0, 0, xc, hc, cur);
    int w0 = 0;  // = ks % 3
    for (int ks = 0; ks < ns; ++ks) {
      const int w1 = w0 == 2 ? 0 : w0 + 1, w2 = w1 == 2 ? 0 : w1 + 1;
      const int zb = ks & 1;
      stg.store(&Xh[w2][0], &Xy[w2][0], tid);  // window of step ks+2 (loaded one step ago)
      float2 h3[NA];
#pragma unroll
      for (int nb = 0; nb < NA; ++nb) h3[nb] = Hrow[nb][hidx(ks + 3)];
      stg.load(a.v, a.vy, tl.cbase + (int64_t)(ks + 3) * KS, tl.tau0, tl.yend, Hrow[0] + hidx(ks + 3), tid);
      build_hankel(w1, zb ^ 1);  // Hankel copies of step ks+1
      load_x(w1, xn);            // samples of step ks+1
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
        Frag nxt;
        if (kb + 1 < NKB)
          fetch(zb, kb + 1, xc, hc, nxt);
        else
          fetch(zb ^ 1, 0, xn, hn, nxt);  // first block of step ks+1
        mma(cur);
        cur = nxt;
      }
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
        for (int g = 0; g < 4; ++g) xc[kb][g] = xn[kb][g];
#pragma unroll
      for (int nb = 0; nb < NA; ++nb) {
        hc[nb] = hn[nb];
        hn[nb] = hnn[nb];
        hnn[nb] = h3[nb];
      }
      w0 = w1;
      {
        constexpr int NMF = NKB * RB * 2 * NA * NB;
#pragma unroll
        for (int i = 0; i < NMF; ++i) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
          __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);  // VALU
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // LDS read
        }
      }
    }
  }
  store_tiles<RB, 2 * NA, AW, 0>(a, tl.id, tl.tau0, tl.alpha0, 0, 0, lane, acc);
}

template <int PREC, int SPLIT, int RB, int NA, int KS>
hipError_t launch_rg(const ContractArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((contract_rg<PREC, SPLIT, RB, NA, KS>), dim3(grid), dim3(64), 0, st, a);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------- register-B contraction, shared Hankel copies
//
// BF16/FP16 tile of TW = 16 RB lags and NW blocks of 32 cycle frequencies, one
// block per wave.  Each wave generates the modulated operands of its own
// cycle frequencies (both tables) directly in the registers of the
// matrix-core B fragments, so they never pass through LDS; the Hankel copies
// are built once per workgroup and step by all threads and shared by the
// waves, so LDS carries only the sample window, the copies and their
// fragment reads.  Same operands and K order as contract_16_tile, so the
// tables are bit-identical.  One barrier per K step.
template <int PREC, int SPLIT, int RB, int NW, int KS, int IL, int PF>
__device__ __forceinline__ void contract_16r_tile(const ContractArgs& a, TileId tid_in) {
  using O = Op<PREC>;
  constexpr int NT = 64 * NW;
  constexpr int TW = 16 * RB, AW = 32 * NW;
  static_assert(KS % 8 == 0, "shape");
  constexpr int NKB = KS / 8;                    // 8-sample K blocks per step
  constexpr int ZW = KS + TW;
  constexpr int ZP = ((ZW + 55) / 64) * 64 + 8;  // layout of contract_16_tile
  constexpr int CO = 4 * ZP;
  constexpr int ZS = CO + 4 * ZP;
  constexpr int XW = ZW + 4;
  constexpr int ZU = ZW;
  constexpr int NB = SPLIT ? 2 : 1;

  __shared__ __attribute__((aligned(16))) uint32_t Zs[2][ZS];
  __shared__ __attribute__((aligned(16))) float2 Xh[2][XW];
  __shared__ __attribute__((aligned(16))) float2 Xy[3][KS];
  __shared__ __attribute__((aligned(16))) float2 Hs[PF == 2 ? 3 : 1][PF == 2 ? NT : 1];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  const Tile tl(a, tid_in, TW, AW, KS);
  const int ns = tl.ns;

  // the lane's cycle frequency and the chunk-relative twiddles of the samples
  // it modulates: j = 8 kb + 4 h + g within a step
  const int al = tl.alpha0 + 32 * w + l32;
  const bool aok = al < a.A;
  float2 lo[NKB][4];
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int g = 0; g < 4; ++g)
      lo[kb][g] = aok ? a.Lo[(int64_t)al * KS + 8 * kb + 4 * h + g] : make_float2(0.f, 0.f);
  const float2* Hcol = a.H + (aok ? al : 0);
  auto hptr = [&](int ks) { return Hcol + (int64_t)min(ks, tl.nsteps - 1) * a.hs; };

  // Hankel fragment of row block rb at K block kb: word zoff0 + 16 rb + 8 kb
  int zoff0;
  {
    const int p0 = (l32 >> 1) + 4 * h;
    const int sh = p0 & 3;
    zoff0 = (l32 & 1) * CO + sh * ZP + (p0 - sh);
  }

  auto build_hankel = [&](int buf) { build_copies<O, NT, ZU, ZP, CO>(&Xh[buf][0], &Zs[buf][0], tid); };

  // modulated fragments of one K block: [b][0] table R (Y), [b][1] table Rc (Yc)
  typedef uint4 BFrag[NB][2];
  auto gen_b = [&](int buf, int kb, float2 hv, BFrag& f) {
    const float4 xa = *reinterpret_cast<const float4*>(&Xy[buf][8 * kb + 4 * h]);
    const float4 xb = *reinterpret_cast<const float4*>(&Xy[buf][8 * kb + 4 * h + 2]);
    const float2 xs[4] = {make_float2(xa.x, xa.y), make_float2(xa.z, xa.w), make_float2(xb.x, xb.y),
                          make_float2(xb.z, xb.w)};
    float2 y[4], yc[4];
    modulate<4>(xs, hv, lo[kb], y, yc);
    uint32_t py[NB][4], pyc[NB][4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      py[0][g] = O::pack(y[g].x, y[g].y);
      pyc[0][g] = O::pack(yc[g].x, yc[g].y);
      if (SPLIT) {
        py[NB - 1][g] = O::pack(y[g].x - O::rnd(y[g].x), y[g].y - O::rnd(y[g].y));
        pyc[NB - 1][g] = O::pack(yc[g].x - O::rnd(yc[g].x), yc[g].y - O::rnd(yc[g].y));
      }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      f[b][0] = make_uint4(py[b][0], py[b][1], py[b][2], py[b][3]);
      f[b][1] = make_uint4(pyc[b][0], pyc[b][1], pyc[b][2], pyc[b][3]);
    }
  };

  f32x16 acc[RB][2];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][k][v] = 0.f;

  // Software pipeline over K blocks: the fragments of the next block (the
  // first block of the next step at a step's end) are generated while the
  // current block's matrix-core instructions run, in two register sets that
  // alternate (NKB is even, so every step starts in set 0).  Hankel fragment
  // (rb, kb) equals (rb + 1, kb - 2), so a step reads its 2 (RB - 1) + NKB
  // distinct ones once.  The samples a lane modulates are read from a
  // triple-buffered Xy: a wave may still read step ks's samples while
  // another writes step ks + 2's.
  static_assert(NKB % 2 == 0, "two fragment sets");
  // the matrix-core work of step ks on Zs[zb] with the next K block's
  // fragments generated in between (from Xy[ycur], or at the step's last
  // block the next step's first one from Xy[ynext])
  BFrag bf[2];
  // The next step's first NCF Hankel fragments are this step's last NCF (its
  // window starts KS samples on): they stay in registers.  Only in the
  // 64-lag waves: the 128-lag ones (one wave per SIMD) read every fragment of
  // a step from LDS, as they did before the carry (with it, the FP16 form of
  // that tile gave non-finite tables in the configuration parity test, cause
  // not found, so it is not used there).
  constexpr int NAF = 2 * (RB - 1) + NKB;
  constexpr int NCF = RB <= 4 ? 2 * (RB - 1) : 0;
  uint4 afc[NCF > 0 ? NCF : 1];
  auto load_carry = [&](int zb) {
    const uint32_t* zp = &Zs[zb][0] + zoff0;
#pragma unroll
    for (int o = 0; o < NCF; ++o) afc[o] = *reinterpret_cast<const uint4*>(zp + 8 * o);
  };
  auto mfma_step = [&](int zb, int ycur, int ynext, float2 hcur, float2 hnext, bool more) {
    const uint32_t* zp = &Zs[zb][0] + zoff0;
    uint4 af[NAF];
#pragma unroll
    for (int o = 0; o < NCF; ++o) af[o] = afc[o];
#pragma unroll
    for (int o = NCF; o < NAF; ++o) af[o] = *reinterpret_cast<const uint4*>(zp + 8 * o);
#pragma unroll
    for (int o = 0; o < NCF; ++o) afc[o] = af[NKB + o];
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
      BFrag& cur = bf[kb & 1];
      BFrag& nxt = bf[(kb & 1) ^ 1];
      if (kb + 1 < NKB)
        gen_b(ycur, kb + 1, hcur, nxt);
      else if (more)
        gen_b(ynext, 0, hnext, nxt);
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          acc[rb][0] = O::mfma(af[2 * rb + kb], cur[b][0], acc[rb][0]);
          acc[rb][1] = O::mfma(af[2 * rb + kb], cur[b][1], acc[rb][1]);
        }
    }
    if (IL) {
      constexpr int NMF = NKB * RB * 2 * NB;
#pragma unroll
      for (int i = 0; i < NMF; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
        __builtin_amdgcn_sched_group_barrier(0x002, IL, 0);  // VALU
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS read
      }
    }
  };
  if (ns > 0 && PF == 1) {
    Stager<NT, XW, KS> stg;
    stg.load(a.v, a.vy, tl.cbase, tl.tau0, tl.yend, hptr(0), tid);
    stg.store(&Xh[0][0], &Xy[0][0], tid);
    float2 hcur = stg.hv;
    stg.load(a.v, a.vy, tl.cbase + KS, tl.tau0, tl.yend, hptr(1), tid);
    stg.store(&Xh[1][0], &Xy[1][0], tid);
    float2 hnext = stg.hv;
    __syncthreads();
    build_hankel(0);
    gen_b(0, 0, hcur, bf[0]);
    __syncthreads();
    load_carry(0);
    int y0 = 0;  // = ks % 3
    for (int ks = 0; ks < ns; ++ks) {
      const int zb = ks & 1;
      const int y1 = y0 == 2 ? 0 : y0 + 1, y2 = y1 == 2 ? 0 : y1 + 1;
      const bool more = ks + 1 < ns;
      if (more)
        stg.load(a.v, a.vy, tl.cbase + (int64_t)(ks + 2) * KS, tl.tau0, tl.yend, hptr(ks + 2), tid);
      mfma_step(zb, y0, y1, hcur, hnext, more);
      if (more) {
        build_hankel(zb ^ 1);                    // step ks + 1 from Xh[zb ^ 1]
        stg.store(&Xh[zb][0], &Xy[y2][0], tid);  // step ks + 2
        hcur = hnext;
        hnext = stg.hv;
        __syncthreads();
      }
      y0 = y1;
    }
  }
  if (ns > 0 && PF == 2) {
    // Loads run two steps ahead in two alternating stagers; the twiddle entry
    // of a step waits in LDS next to its samples (Hs[ks % 3][tid]), so no
    // loaded register is carried across the unrolled loop body.
    Stager<NT, XW, KS> sa, sb;
    sa.load(a.v, a.vy, tl.cbase, tl.tau0, tl.yend, hptr(0), tid);
    sa.store(&Xh[0][0], &Xy[0][0], tid);
    Hs[0][tid] = sa.hv;
    sb.load(a.v, a.vy, tl.cbase + KS, tl.tau0, tl.yend, hptr(1), tid);
    sb.store(&Xh[1][0], &Xy[1][0], tid);
    Hs[1][tid] = sb.hv;
    sa.load(a.v, a.vy, tl.cbase + 2 * KS, tl.tau0, tl.yend, hptr(2), tid);
    __syncthreads();
    build_hankel(0);
    gen_b(0, 0, Hs[0][tid], bf[0]);
    __syncthreads();
    load_carry(0);
    int y0 = 0;  // = ks % 3
    auto body = [&](int ks, Stager<NT, XW, KS>& cur, Stager<NT, XW, KS>& nxt) {
      const int zb = ks & 1;
      const int y1 = y0 == 2 ? 0 : y0 + 1, y2 = y1 == 2 ? 0 : y1 + 1;
      const bool more = ks + 1 < ns;
      if (more)
        nxt.load(a.v, a.vy, tl.cbase + (int64_t)(ks + 3) * KS, tl.tau0, tl.yend, hptr(ks + 3), tid);
      mfma_step(zb, y0, y1, Hs[y0][tid], Hs[y1][tid], more);
      if (more) {
        build_hankel(zb ^ 1);                    // step ks + 1 from Xh[zb ^ 1]
        cur.store(&Xh[zb][0], &Xy[y2][0], tid);  // step ks + 2
        Hs[y2][tid] = cur.hv;
        __syncthreads();
      }
      y0 = y1;
    };
    int ks = 0;
    for (; ks + 1 < ns; ks += 2) {
      body(ks, sa, sb);
      body(ks + 1, sb, sa);
    }
    if (ks < ns) body(ks, sa, sb);
  }
  store_tiles<RB, 2, 32, 0>(a, tl.id, tl.tau0, tl.alpha0 + 32 * w, 0, 0, lane, acc);
}

template <int PREC, int SPLIT, int RB, int NW, int KS, int IL, int PF>
__global__ __launch_bounds__(64 * NW, RB > 4 ? 1 : 2) void contract_16r(ContractArgs a) {
  contract_16r_tile<PREC, SPLIT, RB, NW, KS, IL, PF>(a, tile_of(a));
}

template <int PREC, int SPLIT, int RB, int NW, int KS, int IL, int PF>
__global__ __launch_bounds__(64 * NW, RB > 4 ? 1 : 2) void contract_16r_batch(BatchArgs b) {
  for (;;) {
    const int it = next_item(b.counter);
    if (it >= *b.n_items) break;
    const BItem bi = b.items[it];
    const BJob j = b.jobs[bi.job];
    TileId id;
    id.chunk = 0;
    id.tt = bi.tt;
    id.at = bi.at;
    contract_16r_tile<PREC, SPLIT, RB, NW, KS, IL, PF>(job_args(b, j), id);
  }
}

template <int PREC, int SPLIT, int RB, int NW, int KS, int IL, int PF>
hipError_t launch_16r(const ContractArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((contract_16r<PREC, SPLIT, RB, NW, KS, IL, PF>), dim3(grid), dim3(64 * NW), 0, st, a);
  return hipGetLastError();
}

template <int PREC, int SPLIT, int RB, int NW, int KS, int IL, int PF>
hipError_t launch_16r_batch(const BatchArgs& b, int grid, hipStream_t st) {
  hipLaunchKernelGGL((contract_16r_batch<PREC, SPLIT, RB, NW, KS, IL, PF>), dim3(grid), dim3(64 * NW), 0, st, b);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------- config table

template <int TW, int AW, int WAVES_M, int WAVES_N, int KS, int TBL = 0>
hipError_t launch_f32(const ContractArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((contract_f32<TW, AW, WAVES_M, WAVES_N, KS, TBL>), dim3(grid),
                     dim3(64 * WAVES_M * WAVES_N), 0, st, a);
  return hipGetLastError();
}

template <int PREC, int SPLIT, int TW, int AW, int WAVES_M, int WAVES_N, int KS, int SCHED, int TBL = 0>
hipError_t launch_16(const ContractArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((contract_16<PREC, SPLIT, TW, AW, WAVES_M, WAVES_N, KS, SCHED, TBL>), dim3(grid),
                     dim3(64 * WAVES_M * WAVES_N), 0, st, a);
  return hipGetLastError();
}

template <int TW, int AW, int WAVES_M, int WAVES_N, int KS>
hipError_t launch_f32_batch(const BatchArgs& b, int grid, hipStream_t st) {
  hipLaunchKernelGGL((contract_f32_batch<TW, AW, WAVES_M, WAVES_N, KS>), dim3(grid),
                     dim3(64 * WAVES_M * WAVES_N), 0, st, b);
  return hipGetLastError();
}
template <int PREC, int SPLIT, int TW, int AW, int WAVES_M, int WAVES_N, int KS, int SCHED>
hipError_t launch_16_batch(const BatchArgs& b, int grid, hipStream_t st) {
  hipLaunchKernelGGL((contract_16_batch<PREC, SPLIT, TW, AW, WAVES_M, WAVES_N, KS, SCHED>),
                     dim3(grid), dim3(64 * WAVES_M * WAVES_N), 0, st, b);
  return hipGetLastError();
}
template <typename K>
int resident_grid(K kernel, int threads) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess)
    return 0;
  return ncu * (per > 0 ? per : 1);
}
template <int TW, int AW, int WAVES_M, int WAVES_N, int KS>
int grid_f32_batch() {
  return resident_grid(contract_f32_batch<TW, AW, WAVES_M, WAVES_N, KS>, 64 * WAVES_M * WAVES_N);
}
template <int PREC, int SPLIT, int RB, int NW, int KS, int IL, int PF>
int grid_16r_batch() {
  return resident_grid(contract_16r_batch<PREC, SPLIT, RB, NW, KS, IL, PF>, 64 * NW);
}
template <int PREC, int SPLIT, int TW, int AW, int WAVES_M, int WAVES_N, int KS, int SCHED>
int grid_16_batch() {
  return resident_grid(contract_16_batch<PREC, SPLIT, TW, AW, WAVES_M, WAVES_N, KS, SCHED>,
                       64 * WAVES_M * WAVES_N);
}

#define CFG_F32(TW, AW, WMW, WNW, KS)                                                       \
  {PREC_F32, 0, TW, AW, KS, 64 * WMW * WNW, &launch_f32<TW, AW, WMW, WNW, KS>,              \
   "f32_t" #TW "_a" #AW "_w" #WMW "x" #WNW "_k" #KS,                                        \
   &launch_f32_batch<TW, AW, WMW, WNW, KS>, &grid_f32_batch<TW, AW, WMW, WNW, KS>}
#define CFG_16(P, PN, SP, TW, AW, WMW, WNW, KS, SC)                                         \
  {P, SP, TW, AW, KS, 64 * WMW * WNW, &launch_16<P, SP, TW, AW, WMW, WNW, KS, SC>,          \
   PN "_s" #SP "_t" #TW "_a" #AW "_w" #WMW "x" #WNW "_k" #KS "_i" #SC,                      \
   &launch_16_batch<P, SP, TW, AW, WMW, WNW, KS, SC>,                                       \
   &grid_16_batch<P, SP, TW, AW, WMW, WNW, KS, SC>}
#define CFG_16_ALL(TW, AW, WMW, WNW, KS, SC)                \
  CFG_16(PREC_BF16, "bf16", 0, TW, AW, WMW, WNW, KS, SC),   \
  CFG_16(PREC_BF16, "bf16", 1, TW, AW, WMW, WNW, KS, SC),   \
  CFG_16(PREC_F16, "f16", 0, TW, AW, WMW, WNW, KS, SC),     \
  CFG_16(PREC_F16, "f16", 1, TW, AW, WMW, WNW, KS, SC)

#define CFG_RG(P, PN, SP, RB, NA, KS)                                                      \
  {P, SP, 16 * RB, 32 * NA, KS, 64, &launch_rg<P, SP, RB, NA, KS>,                           \
   PN "_s" #SP "_t" #RB "x16_a" #NA "x32_reg_k" #KS, nullptr, nullptr}
// One-table tiles (TBL = 1: R, 2: Rc): 2 AW cycle frequencies of one table
// per tile, single states only.
#define CFG_F32_T(TW, AW, WMW, WNW, KS, TBL, TN)                                            \
  {PREC_F32, 0, TW, AW, KS, 64 * WMW * WNW, &launch_f32<TW, AW, WMW, WNW, KS, TBL>,         \
   "f32_t" #TW "_a" #AW "_w" #WMW "x" #WNW "_k" #KS "_" TN, nullptr, nullptr, TBL}
#define CFG_16_T(P, PN, SP, TW, AW, WMW, WNW, KS, SC, TBL, TN)                               \
  {P, SP, TW, AW, KS, 64 * WMW * WNW, &launch_16<P, SP, TW, AW, WMW, WNW, KS, SC, TBL>,     \
   PN "_s" #SP "_t" #TW "_a" #AW "_w" #WMW "x" #WNW "_k" #KS "_i" #SC "_" TN, nullptr, nullptr, TBL}
#define CFG_T_ALL(TW, AW, WMW, WNW, TBL, TN)                                        \
  CFG_F32_T(TW, AW, WMW, WNW, 16, TBL, TN),                                         \
  CFG_16_T(PREC_BF16, "bf16", 0, TW, AW, WMW, WNW, 32, 0, TBL, TN),                 \
  CFG_16_T(PREC_BF16, "bf16", 1, TW, AW, WMW, WNW, 32, 0, TBL, TN),                 \
  CFG_16_T(PREC_F16, "f16", 0, TW, AW, WMW, WNW, 32, 0, TBL, TN),                   \
  CFG_16_T(PREC_F16, "f16", 1, TW, AW, WMW, WNW, 32, 0, TBL, TN)

#define CFG_16R(P, PN, SP, RB, NW, KS, IL, PF)                                            \
  {P, SP, 16 * RB, 32 * NW, KS, 64 * NW, &launch_16r<P, SP, RB, NW, KS, IL, PF>,            \
   PN "_s" #SP "_t" #RB "x16_a" #NW "x32_regsh_k" #KS "_i" #IL "_p" #PF,                    \
   &launch_16r_batch<P, SP, RB, NW, KS, IL, PF>, &grid_16r_batch<P, SP, RB, NW, KS, IL, PF>, 0}
#define CFG_16R_ALL(RB, NW, KS, IL, PF)                 \
  CFG_16R(PREC_BF16, "bf16", 0, RB, NW, KS, IL, PF),    \
  CFG_16R(PREC_BF16, "bf16", 1, RB, NW, KS, IL, PF),    \
  CFG_16R(PREC_F16, "f16", 0, RB, NW, KS, IL, PF),      \
  CFG_16R(PREC_F16, "f16", 1, RB, NW, KS, IL, PF)

#define CFG_RG_ALL(RB, NA, KS)                  \
  CFG_RG(PREC_BF16, "bf16", 0, RB, NA, KS),     \
  CFG_RG(PREC_BF16, "bf16", 1, RB, NA, KS),     \
  CFG_RG(PREC_F16, "f16", 0, RB, NA, KS),       \
  CFG_RG(PREC_F16, "f16", 1, RB, NA, KS)

// The first configuration of each (precision, split, lag tile) is the default.
static const KernelCfg g_cfgs[] = {
    CFG_F32(128, 64, 4, 1, 16),
    CFG_F32(64, 64, 2, 1, 16),
    CFG_F32(32, 64, 1, 2, 16),
    CFG_F32(64, 128, 2, 2, 16),
    CFG_F32(64, 64, 2, 2, 16),
    CFG_16_ALL(128, 64, 4, 1, 32, 0),
    CFG_16_ALL(64, 64, 2, 1, 32, 0),
    CFG_16_ALL(32, 64, 1, 2, 32, 0),
    CFG_16_ALL(64, 128, 2, 2, 32, 0),
    CFG_16_ALL(128, 64, 4, 1, 32, 1),
    CFG_16_ALL(128, 128, 4, 2, 32, 0),
    CFG_16_ALL(128, 128, 4, 2, 32, 1),
    CFG_16_ALL(128, 128, 2, 2, 32, 1),
    CFG_16_ALL(64, 64, 2, 2, 32, 0),
    CFG_RG_ALL(8, 1, 32),
    CFG_16R_ALL(4, 4, 32, 0, 2),
    CFG_16R_ALL(4, 4, 32, 6, 1),
    CFG_16R_ALL(4, 4, 32, 0, 1),
    CFG_16R_ALL(4, 2, 32, 0, 1),
    CFG_16R_ALL(8, 4, 32, 0, 1),
    CFG_16_ALL(128, 64, 2, 2, 32, 1),
    CFG_16_ALL(128, 64, 2, 2, 32, 0),
    CFG_16_ALL(64, 64, 2, 2, 32, 8),
    CFG_16_ALL(64, 64, 2, 2, 32, 6),
    CFG_T_ALL(128, 64, 4, 1, 1, "R"),
    CFG_T_ALL(64, 64, 2, 1, 1, "R"),
    CFG_T_ALL(32, 64, 1, 2, 1, "R"),
    CFG_T_ALL(128, 64, 4, 1, 2, "Rc"),
    CFG_T_ALL(64, 64, 2, 1, 2, "Rc"),
    CFG_T_ALL(32, 64, 1, 2, 2, "Rc"),
};

const KernelCfg* kernel_cfgs(int* n) {
  *n = (int)(sizeof(g_cfgs) / sizeof(g_cfgs[0]));
  return g_cfgs;
}

// ----------------------------------------------------------------------------- small kernels

// Lo[a][k] = exp(-j2pi frac(alpha_a k)), k < ks;  H[s][a] = exp(-j2pi frac(alpha_a s ks)) (rows of
// A cycle frequencies, so the per-step loads of a tile are coalesced).
__global__ void tables_kernel(const double* alpha_r, int A, int ks, int nsteps, float2* Lo,
                              float2* H) {
  const int64_t per = ks + nsteps;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)A * per) return;
  const int a = (int)(i / per), k = (int)(i % per);
  const int64_t n = k < ks ? (int64_t)k : (int64_t)(k - ks) * ks;
  double s, c;
  sincospi(2.0 * frac_prod(alpha_r[a], n), &s, &c);
  const float2 w = make_float2((float)c, (float)-s);
  if (k < ks)
    Lo[(int64_t)a * ks + k] = w;
  else
    H[(int64_t)(k - ks) * A + a] = w;
}

// E[c][a] = exp(-j2pi frac(alpha_a (base0 + c Kc))) in FP64 (absolute sample index).
__global__ void phase_kernel(const double* alpha_r, int A, int64_t base0, int Kc, int nc,
                             double2* E) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nc * A) return;
  const int c = (int)(i / A), a = (int)(i % A);
  double s, co;
  sincospi(2.0 * frac_prod(alpha_r[a], base0 + (int64_t)c * Kc), &s, &co);
  E[i] = make_double2(co, -s);
}

// S += sum_c part[c] * E[c] in FP64, chunks in ascending order (first: S starts at 0).
__global__ void accumulate_kernel(double2* S, const float2* part, const double2* E, int T, int A,
                                  int nc, int first, int tbl) {
  const int64_t n2 = 2 * (int64_t)T * A;
  // tbl 0: both tables; 1 / 2: only the elements of table R / Rc
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + (tbl ? (int64_t)(tbl - 1) * T * A : 0);
  if (i >= (tbl ? (int64_t)tbl * T * A : n2)) return;
  const int a = (int)(i % A);
  double2 s = first ? make_double2(0.0, 0.0) : S[i];
  for (int c = 0; c < nc; ++c) {
    const float2 p = part[(int64_t)c * n2 + i];
    const double2 e = E[(int64_t)c * A + a];
    const double pr = p.x, pi = p.y;
    s.x += pr * e.x - pi * e.y;
    s.y += pr * e.y + pi * e.x;
  }
  S[i] = s;
}

// out[t][a] = (S + part0 * E0) / n_used for both tables.
template <int C128>
__global__ void finalize_kernel(const double2* S, int hasS, const float2* part0, const double2* E0,
                                int hasP, int T, int A, double nd, void* R, void* Rc) {
  const int64_t TA = (int64_t)T * A;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * TA) return;
  const int table = i >= TA ? 1 : 0;
  void* out = table ? Rc : R;
  if (out == nullptr) return;
  const int64_t r = i - table * TA;
  const int a = (int)(r % A);
  double sr = 0.0, si = 0.0;
  if (hasS) {
    const double2 s = S[i];
    sr = s.x;
    si = s.y;
  }
  if (hasP) {
    const float2 p = part0[i];
    const double2 e = E0[a];
    const double pr = p.x, pi = p.y;
    sr += pr * e.x - pi * e.y;
    si += pr * e.y + pi * e.x;
  }
  sr /= nd;
  si /= nd;
  if (C128)
    reinterpret_cast<double2*>(out)[r] = make_double2(sr, si);
  else
    reinterpret_cast<float2*>(out)[r] = make_float2((float)sr, (float)si);
}

__global__ void vcopy_kernel(VSrc v, int64_t shift, int64_t n, float2* dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = vload(v, shift + i);
}

// Deterministic unit-magnitude test samples for the autotuner's timing runs.
__global__ void pattern_kernel(float2* x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    float s, c;
    __sincosf(0.001f * (float)(i % 100003) + 0.3f * (float)(i % 7), &s, &c);
    x[i] = make_float2(c, s);
  }
}

hipError_t launch_pattern(float2* x, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(pattern_kernel, dim3((int)((n + 255) / 256)), dim3(256), 0, st, x, n);
  return hipGetLastError();
}

__global__ void zero_kernel(uint32_t* p, int64_t nwords) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nwords) p[i] = 0u;
}

// ---- batched small kernels (grid-stride over device-resident descriptors) --

__global__ void batch_reset_kernel(int* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

__global__ void batch_phase_kernel(const BJob* jobs, const BCounts* cnt) {
  const int nj = cnt->n_jobs;
  for (int j = blockIdx.x; j < nj; j += gridDim.x) {
    const BJob jb = jobs[j];
    for (int a = threadIdx.x; a < jb.A; a += blockDim.x) {
      double s, c;
      sincospi(2.0 * frac_prod(jb.alpha_r[a], jb.abs_base), &s, &c);
      jb.E[a] = make_double2(c, -s);
    }
  }
}

__global__ void batch_accumulate_kernel(const BJob* jobs, const BAcc* acc, const BTile* tiles,
                                        const BCounts* cnt) {
  const int nt = cnt->n_acc_tiles;
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    const BTile tl = tiles[t];
    const BAcc d = acc[tl.desc];
    const int64_t i = tl.off + threadIdx.x;
    if (i >= d.n2) continue;
    const int a = (int)(i % d.A);
    double2 s = d.first ? make_double2(0.0, 0.0) : d.S[i];
    for (int c = 0; c < d.njobs; ++c) {
      const BJob& jb = jobs[d.job0 + c];
      const float2 p = jb.part[i];
      const double2 e = jb.E[a];
      const double pr = p.x, pi = p.y;
      s.x += pr * e.x - pi * e.y;
      s.y += pr * e.y + pi * e.x;
    }
    d.S[i] = s;
  }
}

__global__ void batch_copy_kernel(const BCopy* copies, const BTile* tiles, const BCounts* cnt) {
  const int nt = cnt->n_copy_tiles;
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    const BTile tl = tiles[t];
    const BCopy d = copies[tl.desc];
    const int64_t i = tl.off + threadIdx.x;
    if (i < d.n) d.dst[i] = vload(d.v, d.shift + i);
  }
}

__global__ void batch_finalize_kernel(const BJob* jobs, const BFin* fin, const BTile* tiles,
                                      const BCounts* cnt) {
  const int nt = cnt->n_fin_tiles;
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    const BTile tl = tiles[t];
    const BFin d = fin[tl.desc];
    const int64_t i = tl.off + threadIdx.x;
    if (i >= 2 * d.TA) continue;
    const int table = i >= d.TA ? 1 : 0;
    void* out = table ? d.Rc : d.R;
    if (out == nullptr) continue;
    const int64_t r = i - table * d.TA;
    const int a = (int)(r % d.A);
    double sr = 0.0, si = 0.0;
    if (d.hasS) {
      const double2 sv = d.S[i];
      sr = sv.x;
      si = sv.y;
    }
    if (d.job >= 0) {
      const BJob& jb = jobs[d.job];
      const float2 p = jb.part[i];
      const double2 e = jb.E[a];
      const double pr = p.x, pi = p.y;
      sr += pr * e.x - pi * e.y;
      si += pr * e.y + pi * e.x;
    }
    sr /= d.nd;
    si /= d.nd;
    if (d.c128)
      reinterpret_cast<double2*>(out)[r] = make_double2(sr, si);
    else
      reinterpret_cast<float2*>(out)[r] = make_float2((float)sr, (float)si);
  }
}

// stage 0: counter reset + phases (before the contraction);
// stage 1: accumulation + pending-sample copies (after it).
hipError_t launch_batch_small(const BJob* jobs, const BCounts* cnt, const BAcc* acc,
                              const BTile* acc_tiles, const BCopy* copies,
                              const BTile* copy_tiles, int* counter, int stage,
                              hipStream_t st) {
  if (stage == 0) {
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, st, counter);
    hipLaunchKernelGGL(batch_phase_kernel, dim3(1024), dim3(256), 0, st, jobs, cnt);
  } else {
    hipLaunchKernelGGL(batch_accumulate_kernel, dim3(4096), dim3(256), 0, st, jobs, acc, acc_tiles,
                       cnt);
    hipLaunchKernelGGL(batch_copy_kernel, dim3(1024), dim3(256), 0, st, copies, copy_tiles, cnt);
  }
  return hipGetLastError();
}

hipError_t launch_batch_finalize(const BJob* jobs, const BFin* fin, const BTile* tiles,
                                 const BCounts* cnt, hipStream_t st) {
  hipLaunchKernelGGL(batch_finalize_kernel, dim3(4096), dim3(256), 0, st, jobs, fin, tiles, cnt);
  return hipGetLastError();
}

static inline int nblocks(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

hipError_t launch_tables(const double* alpha_r, int A, int ks, int nsteps, float2* Lo, float2* H,
                         hipStream_t st) {
  const int64_t n = (int64_t)A * (ks + nsteps);
  hipLaunchKernelGGL(tables_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, alpha_r, A, ks,
                     nsteps, Lo, H);
  return hipGetLastError();
}

hipError_t launch_phase(const double* alpha_r, int A, int64_t base0, int Kc, int nc, double2* E,
                        hipStream_t st) {
  const int64_t n = (int64_t)A * nc;
  hipLaunchKernelGGL(phase_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, alpha_r, A, base0, Kc,
                     nc, E);
  return hipGetLastError();
}

hipError_t launch_accumulate(double2* S, const float2* part, const double2* E, int T, int A, int nc,
                             int first, int tbl, hipStream_t st) {
  const int64_t n = (tbl ? 1 : 2) * (int64_t)T * A;
  hipLaunchKernelGGL(accumulate_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, S, part, E, T, A,
                     nc, first, tbl);
  return hipGetLastError();
}

hipError_t launch_finalize(const double2* S, int hasS, const float2* part0, const double2* E0,
                           int hasP, int T, int A, int64_t n_used, void* R, void* Rc, int c128,
                           hipStream_t st) {
  const int64_t n = 2 * (int64_t)T * A;
  if (c128)
    hipLaunchKernelGGL(finalize_kernel<1>, dim3(nblocks(n, 256)), dim3(256), 0, st, S, hasS, part0,
                       E0, hasP, T, A, (double)n_used, R, Rc);
  else
    hipLaunchKernelGGL(finalize_kernel<0>, dim3(nblocks(n, 256)), dim3(256), 0, st, S, hasS, part0,
                       E0, hasP, T, A, (double)n_used, R, Rc);
  return hipGetLastError();
}

hipError_t launch_vcopy(VSrc v, int64_t shift, int64_t n, float2* dst, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(vcopy_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, v, shift, n, dst);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, int64_t bytes, hipStream_t st) {
  const int64_t nw = bytes / 4;
  if (nw <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3(nblocks(nw, 256)), dim3(256), 0, st,
                     reinterpret_cast<uint32_t*>(p), nw);
  return hipGetLastError();
}

}  // namespace cyclo
