// Internal interfaces between the C-ABI runtime and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cyclo {

// Virtual sample array: pend[0 .. n_pend) followed by xin[0 .. n_avail - n_pend).
// Reads at or beyond n_avail return 0.
struct VSrc {
  const float2* pend;
  const float2* xin;
  int64_t n_pend;
  int64_t n_avail;
};

// One launch of the chunk contraction: for chunk c (0 <= c < n_chunks) the
// chunk-local partial sums
//   part[c][0][t][a] = sum_{l < m_c} x[b_c+l+t] conj(x[b_c+l]) W[l][a]
//   part[c][1][t][a] = sum_{l < m_c} x[b_c+l+t]      x[b_c+l]  W[l][a]
// with b_c = v_off + c*Kc (virtual index), m_c = min(Kc, n_prod - c*Kc) and
// the chunk-relative twiddle W[l][a] = H[l / KS][a] * Lo[a][l % KS]
//                                  = exp(-j 2 pi frac(alpha_a l)).
struct ContractArgs {
  VSrc v;   // Hankel (leading) samples: product i, lag t reads v[i + t]
  VSrc vy;  // modulated (trailing) samples: product i reads vy[i]; == v for one input
  int64_t v_off;
  int64_t n_prod;
  int T, A, Kc;
  int n_tt, n_at, n_chunks;
  const float2* H;   // [Kc/KS][hs]: step s of cycle frequency a at H[s * hs + a]
  const float2* Lo;  // [A][KS]
  float2* part;      // [n_chunks][2][T][A]
  int hs;            // row stride of H (>= A)
};

enum { PREC_F32 = 0, PREC_BF16 = 1, PREC_F16 = 2 };

// ---- batched (many stream states, one launch per kernel) ------------------
// One contraction job: one chunk of one stream in one push (or the pending
// partial chunk of one stream in a read).
struct BJob {
  VSrc v;              // the stream's virtual sample array for this call
  int64_t v_off;       // virtual index of the chunk's first product
  int64_t n_prod;      // products in the chunk (<= Kc)
  int64_t abs_base;    // absolute sample index of the chunk's first product
  const double* alpha_r;
  const float2* H;
  const float2* Lo;
  float2* part;        // [2][T][A] chunk partial
  double2* E;          // [A] chunk phase factor
  int A;
  int pad;
};
struct BItem {         // contraction work item
  int job, tt, at, pad;
};
struct BAcc {          // S += sum of the stream's jobs [job0, job0 + njobs) in order
  double2* S;
  int64_t n2;          // 2*T*A
  int job0, njobs, A, first;
};
struct BFin {          // read: out = (S + partial job * E) / n_used
  const double2* S;
  void* R;
  void* Rc;
  int64_t TA;
  double nd;
  int job;             // partial job or -1
  int hasS, A, c128;
};
struct BCopy {         // dst[i] = v[shift + i], i < n
  VSrc v;
  int64_t shift, n;
  float2* dst;
};
struct BTile {         // a block of 256 elements of descriptor `desc`
  int desc, pad;
  int64_t off;
};
// Counts live in device memory so one captured graph serves every call.
struct BCounts {
  int n_jobs, n_items, n_acc_tiles, n_copy_tiles, n_fin_tiles, counter, pad0, pad1;
};
struct BatchArgs {
  const BJob* jobs;
  const BItem* items;
  const int* n_items;
  int* counter;
  int T, Kc;
  int hs;  // row stride of the twiddle table H (all streams' cycle frequencies)
};

typedef hipError_t (*BatchLaunch)(const BatchArgs&, int grid, hipStream_t);

struct KernelCfg {
  int prec;      // PREC_*
  int split;     // modulated operand split into hi + lo
  int tw;        // lags per workgroup tile
  int aw;        // cycle frequencies per workgroup tile
  int ks;        // samples per K step (twiddle table period)
  int nthreads;  // workgroup size
  hipError_t (*launch)(const ContractArgs&, int grid, hipStream_t);
  const char* name;
  // persistent batched form (nullptr if none) and its resident grid size
  BatchLaunch blaunch;
  int (*bgrid)();
  // tables computed: 0 both (tile columns: aw cycle frequencies of R then of
  // Rc), 1 R only or 2 Rc only (tile columns: 2 aw cycle frequencies)
  int tbl;
};

const KernelCfg* kernel_cfgs(int* n);

hipError_t launch_batch_small(const BJob* jobs, const BCounts* cnt, const BAcc* acc,
                              const BTile* acc_tiles, const BCopy* copies,
                              const BTile* copy_tiles, int* counter, int stage,
                              hipStream_t st);
hipError_t launch_batch_finalize(const BJob* jobs, const BFin* fin, const BTile* tiles,
                                 const BCounts* cnt, hipStream_t st);

hipError_t launch_tables(const double* alpha_r, int A, int ks, int nsteps, float2* Lo,
                         float2* H, hipStream_t st);
hipError_t launch_phase(const double* alpha_r, int A, int64_t base0, int Kc, int nc,
                        double2* E, hipStream_t st);
hipError_t launch_accumulate(double2* S, const float2* part, const double2* E, int T, int A,
                             int nc, int first, int tbl, hipStream_t st);
hipError_t launch_finalize(const double2* S, int hasS, const float2* part0, const double2* E0,
                           int hasP, int T, int A, int64_t n_used, void* R, void* Rc, int c128,
                           hipStream_t st);
hipError_t launch_vcopy(VSrc v, int64_t shift, int64_t n, float2* dst, hipStream_t st);
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t st);
hipError_t launch_pattern(float2* x, int64_t n, hipStream_t st);

}  // namespace cyclo
