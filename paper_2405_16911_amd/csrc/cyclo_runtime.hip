// Stream state and C ABI (include/cyclo.h) of the cyclic-statistics library.
//
// State layout in HBM (one stream):
//   alpha_r [A]            FP64 cycle frequencies reduced to [-1/2, 1/2]
//   Lo [A][KS], H [A][Kc/KS]  FP32 chunk-relative twiddle tables
//   S [2][T][A]            FP64 complex accumulators (R, Rc) over committed chunks
//   pend[2][Kc+T-1]        ping-pong buffers of not-yet-committed samples
//   part [maxc][2][T][A]   FP32 complex chunk partials (workspace)
//   E [maxc][A]            FP64 complex per-chunk phase factors (workspace)
//
// Products are committed in chunks aligned to absolute indices [c Kc, (c+1) Kc)
// as soon as their samples are all present, in ascending c, so the committed
// accumulator after L samples does not depend on how the samples were pushed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <cstdio>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/cyclo.h"
#include "cyclo_internal.h"

using namespace cyclo;

namespace cyclo {
hipError_t launch_window_store(double2* ring, const float2* part, const double2* E, int T, int A, int nc,
                               int64_t c0, int W, hipStream_t st);
hipError_t launch_window_finalize(const double2* ring, int W, int s0, int Wn, int T, int A, const double* alpha_r,
                                  int64_t n_ref, int64_t n_used, void* R, void* Rc, int c128, hipStream_t st);
}  // namespace cyclo

struct cyc_state {
  int T = 0, A = 0;
  uint32_t flags = 0;
  int Kc = 0, KS = 0, nsteps = 0;
  int cfg = -1;
  int maxc = 0;
  double* alpha_r = nullptr;
  float2* Lo = nullptr;
  float2* H = nullptr;
  double2* S = nullptr;
  float2* pend[2] = {nullptr, nullptr};   // leading input x, from absolute index nc + dx
  float2* pendy[2] = {nullptr, nullptr};  // trailing input y, from nc + dy (two-input states)
  int cur = 0;
  bool two = false;              // two inputs (cyc_create2)
  int64_t lag_min = 0, dx = 0, dy = 0, lagabs = 0;
  int64_t PC = 0;                // pending capacity (samples)
  int64_t G = 0;                 // a push commits nothing while fewer than G products are pending (0: at once)
  int win = 0;                   // sliding window: hops per window (0: cumulative)
  double2* ring = nullptr;       // [win][2][T][A] FP64 contribution of each hop in the window
  float2* part = nullptr;
  double2* E = nullptr;
  int64_t L = 0;
  int64_t nc = 0;  // products committed
  int tbl = 0;     // tables computed: 0 both, 1 R only, 2 Rc only
  bool poisoned = false;
  // Overlap: the workspace is split in two halves; each push launch contracts
  // into one half on the caller's stream, and the FP64 accumulation of that
  // half runs on `side` while the next launch contracts into the other half.
  // Events order it: ev_part[h] (contraction into h done) -> accumulation of
  // h -> ev_acc[h] (h free again).  side == nullptr: everything on the
  // caller's stream (window states, a one-chunk workspace, CYC_SERIAL_ACC=1).
  hipStream_t side = nullptr;
  hipEvent_t ev_part[2] = {nullptr, nullptr};
  hipEvent_t ev_acc[2] = {nullptr, nullptr};
  bool acc_used[2] = {false, false};
  int half = 0, last_half = -1;
  int maxc_half = 0;
  // contraction-kernel timing
  bool prof = false;
  std::vector<hipEvent_t> ev;  // start/end pairs
  size_t ev_used = 0;
  double prof_work = 0.0;
};

namespace {

constexpr int kMaxLag = 4096;
constexpr int64_t kMaxLagShift = 1 << 20;  // |lag_min| of two-input states

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

int64_t env_i64(const char* name, int64_t dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  char* end = nullptr;
  long long r = std::strtoll(v, &end, 10);
  return (end && *end == 0) ? (int64_t)r : dflt;
}

// ---- tuning cache: (arch, prec, split, T, A-bucket) -> configuration name
typedef std::tuple<std::string, int, int, int, int> TuneKey;
std::mutex g_tune_mu;
std::map<TuneKey, std::string> g_tune;
bool g_tune_loaded = false;

int a_bucket(int A) {
  int b = 0;
  while ((1 << b) < A && b < 30) ++b;
  return b;
}

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

int cfg_by_name(const std::string& name) {
  int n = 0;
  const KernelCfg* c = kernel_cfgs(&n);
  for (int i = 0; i < n; ++i)
    if (name == c[i].name) return i;
  return -1;
}

// Cache file format, one entry per line: "arch prec split T abucket cfg_name".
void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("CYC_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char arch[64], name[128];
  int prec, split, T, ab;
  while (std::fscanf(f, "%63s %d %d %d %d %127s", arch, &prec, &split, &T, &ab, name) == 6)
    g_tune[TuneKey(arch, prec, split, T, ab)] = name;
  std::fclose(f);
}

void tune_store(const TuneKey& k, const std::string& name) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  g_tune[k] = name;
  const char* path = std::getenv("CYC_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %d %s\n", std::get<0>(k).c_str(), std::get<1>(k), std::get<2>(k),
               std::get<3>(k), std::get<4>(k), name.c_str());
  std::fclose(f);
}

// Chooses the contraction kernel for (precision, split, tables, T, A): an
// explicit CYC_KERNEL_CFG index if it implements the mode, else the tuning
// cache, else the first configuration whose lag tile fits T.  The cache keys
// the mode as (prec, split + 2 tbl).
int pick_cfg(int prec, int split, int tbl, int T, int A) {
  int n = 0;
  const KernelCfg* c = kernel_cfgs(&n);
  auto mode_ok = [&](int i) { return c[i].prec == prec && c[i].split == split && c[i].tbl == tbl; };
  const int64_t forced = env_i64("CYC_KERNEL_CFG", -1);
  if (forced >= 0 && forced < n && mode_ok((int)forced)) return (int)forced;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(TuneKey(device_arch(), prec, split + 2 * tbl, T, a_bucket(A)));
    if (it != g_tune.end()) {
      const int i = cfg_by_name(it->second);
      if (i >= 0 && mode_ok(i)) return i;
    }
  }
  const int want_tw = T > 64 ? 128 : (T > 32 ? 64 : 32);
  // 16-bit operands at 33..64 lags: the register-operand tile with shared
  // Hankel copies (the fastest measured there)
  if (prec != PREC_F32 && want_tw == 64)
    for (int i = 0; i < n; ++i)
      if (mode_ok(i) && c[i].tw == 64 && c[i].aw == 128 && c[i].nthreads == 256 && std::strstr(c[i].name, "regsh"))
        return i;
  int best = -1;
  for (int i = 0; i < n; ++i) {
    if (!mode_ok(i) || c[i].tw != want_tw || c[i].aw != 64) continue;
    if (best < 0 || (c[best].nthreads != 256 && c[i].nthreads == 256)) best = i;
  }
  return best;
}

}  // namespace

// Shared with the batch runtime.
int cyc_pick_cfg(int prec, int split, int T, int A) { return pick_cfg(prec, split, 0, T, A); }

namespace {

void free_state(cyc_state* s) {
  if (!s) return;
  for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
  for (int h = 0; h < 2; ++h) {
    if (s->ev_part[h]) (void)hipEventDestroy(s->ev_part[h]);
    if (s->ev_acc[h]) (void)hipEventDestroy(s->ev_acc[h]);
  }
  if (s->side) (void)hipStreamDestroy(s->side);
  (void)hipFree(s->alpha_r);
  (void)hipFree(s->Lo);
  (void)hipFree(s->H);
  (void)hipFree(s->S);
  (void)hipFree(s->pend[0]);
  (void)hipFree(s->pend[1]);
  (void)hipFree(s->pendy[0]);
  (void)hipFree(s->pendy[1]);
  (void)hipFree(s->part);
  (void)hipFree(s->ring);
  (void)hipFree(s->E);
  delete s;
}

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T));
}

int fail_device(cyc_state* s) {
  s->poisoned = true;
  return CYC_EDEVICE;
}

}  // namespace

static hipError_t run_contract(cyc_state* s, const VSrc& v, const VSrc& vy, int64_t v_off, int64_t n_prod,
                               int nch, hipStream_t st, float2* part = nullptr) {
  int ncfg = 0;
  const KernelCfg& cfg = kernel_cfgs(&ncfg)[s->cfg];
  ContractArgs a;
  a.v = v;
  a.vy = vy;
  a.v_off = v_off;
  a.n_prod = n_prod;
  a.T = s->T;
  a.A = s->A;
  a.Kc = s->Kc;
  a.n_tt = (s->T + cfg.tw - 1) / cfg.tw;
  const int atile = cfg.tbl ? 2 * cfg.aw : cfg.aw;  // cycle frequencies per tile
  a.n_at = (s->A + atile - 1) / atile;
  a.n_chunks = nch;
  a.H = s->H;
  a.hs = s->A;
  a.Lo = s->Lo;
  a.part = part ? part : s->part;
  const int64_t grid = (int64_t)a.n_tt * a.n_at * nch;
  if (grid <= 0 || grid > 0x7fffffff) return hipErrorInvalidValue;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (s->prof) {
    while (s->ev.size() < s->ev_used + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return hipErrorOutOfMemory;
      s->ev.push_back(e);
    }
    e0 = s->ev[s->ev_used];
    e1 = s->ev[s->ev_used + 1];
    s->ev_used += 2;
    s->prof_work += (double)n_prod * s->T * s->A;
    hipError_t r = hipEventRecord(e0, st);
    if (r != hipSuccess) return r;
  }
  hipError_t r = cfg.launch(a, (int)grid, st);
  if (r == hipSuccess && e1) r = hipEventRecord(e1, st);
  return r;
}

extern "C" {

const char* cyc_status_str(int code) {
  switch (code) {
    case CYC_OK: return "ok";
    case CYC_EINVAL: return "invalid argument";
    case CYC_ENOMEM: return "out of memory";
    case CYC_EDEVICE: return "device error (state poisoned)";
    case CYC_ESTATE: return "state poisoned by an earlier device error; call cyc_reset";
    case CYC_EUNSUPPORTED: return "unsupported flag combination or size";
    default: return "unknown status code";
  }
}

static int create_state(cyc_state** out, const double* alphas_host, int32_t n_alpha, int64_t lag_min,
                        int32_t n_lag, uint32_t flags, bool two, int32_t hop, int32_t n_hops, void* stream) {
  if (!out || !alphas_host || n_alpha < 1 || n_lag < 1 || n_lag > kMaxLag) return CYC_EINVAL;
  if (n_hops < 0 || n_hops > 4096 || (n_hops > 0 && (hop < 32 || hop > (1 << 20) || hop % 32 != 0)))
    return CYC_EINVAL;
  if (lag_min < -kMaxLagShift || lag_min > kMaxLagShift) return CYC_EINVAL;
  if (flags & ~(CYC_OP_MASK | CYC_TW_SPLIT | CYC_OUT_C128 | CYC_TBL_R | CYC_TBL_RCONJ)) return CYC_EINVAL;
  const int prec = (int)(flags & CYC_OP_MASK);
  if (prec == 3) return CYC_EINVAL;
  const int split = (flags & CYC_TW_SPLIT) ? 1 : 0;
  if (split && prec == PREC_F32) return CYC_EUNSUPPORTED;
  const bool want_r = flags & CYC_TBL_R, want_rc = flags & CYC_TBL_RCONJ;
  const int tbl = want_r == want_rc ? 0 : (want_r ? 1 : 2);
  if (tbl && n_hops > 0) return CYC_EUNSUPPORTED;  // the window form keeps both tables
  for (int32_t i = 0; i < n_alpha; ++i)
    if (!std::isfinite(alphas_host[i])) return CYC_EINVAL;

  cyc_state* s = new (std::nothrow) cyc_state();
  if (!s) return CYC_ENOMEM;
  s->T = n_lag;
  s->A = n_alpha;
  s->flags = flags;
  s->two = two;
  s->lag_min = lag_min;
  s->dx = std::max<int64_t>(0, lag_min);
  s->dy = std::max<int64_t>(0, -lag_min);
  s->lagabs = lag_min < 0 ? -lag_min : lag_min;
  s->tbl = tbl;
  s->cfg = pick_cfg(prec, split, tbl, n_lag, n_alpha);
  if (s->cfg < 0) {
    delete s;
    return CYC_EUNSUPPORTED;
  }
  int ncfg = 0;
  const KernelCfg& cfg = kernel_cfgs(&ncfg)[s->cfg];
  s->KS = cfg.ks;
  // Push coalescing: with 16-bit operands a 2^16-sample push is only a few
  // hundred microseconds of contraction, so a cumulative state lets pushes
  // pile up until 2^18 products are pending (CYC_COALESCE, read at creation;
  // 0 commits at every push) and contracts them in one launch.  Chunks stay
  // aligned to absolute product indices and are committed in ascending order,
  // so results do not change; a read commits whatever is still pending.
  const int64_t coal = (prec != PREC_F32 && n_hops == 0)
                           ? std::max<int64_t>(0, std::min<int64_t>(env_i64("CYC_COALESCE", 1 << 18), 1 << 24))
                           : 0;
  // Products per FP32-accumulated chunk.  A launch's work is split over
  // (tiles x chunks); FP32 keeps 4096.  With 16-bit operands a longer chunk
  // halves or quarters the FP32 partials written per product (and the FP64
  // accumulation that reads them), which pays while one launch (the
  // coalescing target, else a 2^16-sample push) still gives at least two
  // workgroups per CU: 16384 from 32 lag-by-alpha tiles on 256 CUs with the
  // 2^18 target (128 without coalescing), 8192 from 16 (64), else 4096.
  // (Batches take 16384: their streams supply the parallelism.)
  int64_t kc_def = 4096;
  if (prec != PREC_F32 && n_hops == 0) {
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
      ncu = 256;
    const int64_t tiles = (int64_t)((s->A + cfg.aw - 1) / cfg.aw) * ((s->T + cfg.tw - 1) / cfg.tw);
    const int64_t launch = coal > 0 ? coal : 65536;
    if (tiles * (launch / 16384) >= 2 * (int64_t)ncu)
      kc_def = 16384;
    else if (tiles * (launch / 8192) >= 2 * (int64_t)ncu)
      kc_def = 8192;
  }
  int64_t kc = n_hops > 0 ? hop : env_i64("CYC_CHUNK", kc_def);
  kc = std::max<int64_t>(cfg.ks, std::min<int64_t>(kc, 1 << 20));
  kc = (kc / cfg.ks) * cfg.ks;
  s->Kc = (int)kc;
  s->nsteps = s->Kc / s->KS;
  s->win = n_hops;
  s->G = coal > 0 ? std::max<int64_t>(kc, (coal + kc - 1) / kc * kc) : 0;
  // pending samples of either input: < max(Kc, G) products plus T - 1 + |lag_min| samples
  s->PC = std::max<int64_t>(s->Kc, s->G) + s->T + s->lagabs;

  const int64_t TA2 = 2 * (int64_t)s->T * s->A;
  // Partial-sum workspace: room for eight chunks' FP32 partials (four per half
  // of the overlapped push), within 256 MiB .. 2 GiB, so a large table still
  // contracts a whole 2^16-sample push in one launch (at 64 lags x 65536
  // cycle frequencies a chunk's partials are 64 MiB).
  const int64_t ws_def_mb = std::max<int64_t>(256, std::min<int64_t>(2048, (8 * TA2 * 8 + (1 << 20) - 1) >> 20));
  const int64_t ws_bytes = env_i64("CYC_WORKSPACE_MB", ws_def_mb) << 20;
  s->maxc = (int)std::max<int64_t>(1, std::min<int64_t>(4096, ws_bytes / (TA2 * 8)));

  hipStream_t st = as_stream(stream);
  // alpha reduced to [-1/2, 1/2]: the tables are 1-periodic in alpha and the
  // reduction alpha - rint(alpha) is exact in FP64.
  double* ar = new (std::nothrow) double[n_alpha];
  if (!ar) {
    delete s;
    return CYC_ENOMEM;
  }
  for (int32_t i = 0; i < n_alpha; ++i) ar[i] = alphas_host[i] - std::nearbyint(alphas_host[i]);

  int rc = CYC_OK;
  if (dalloc(&s->alpha_r, s->A) != hipSuccess || dalloc(&s->Lo, (size_t)s->A * s->KS) != hipSuccess ||
      dalloc(&s->H, (size_t)s->A * s->nsteps) != hipSuccess || dalloc(&s->S, (size_t)TA2) != hipSuccess ||
      dalloc(&s->pend[0], (size_t)s->PC) != hipSuccess || dalloc(&s->pend[1], (size_t)s->PC) != hipSuccess ||
      (two && (dalloc(&s->pendy[0], (size_t)s->PC) != hipSuccess ||
               dalloc(&s->pendy[1], (size_t)s->PC) != hipSuccess)) ||
      dalloc(&s->part, (size_t)s->maxc * TA2) != hipSuccess ||
      (s->win > 0 && dalloc(&s->ring, (size_t)s->win * TA2) != hipSuccess) ||
      dalloc(&s->E, (size_t)s->maxc * s->A) != hipSuccess) {
    rc = CYC_ENOMEM;
  }
  if (rc == CYC_OK) {
    if (hipMemcpyAsync(s->alpha_r, ar, sizeof(double) * s->A, hipMemcpyHostToDevice, st) != hipSuccess ||
        launch_tables(s->alpha_r, s->A, s->KS, s->nsteps, s->Lo, s->H, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      rc = CYC_EDEVICE;
  }
  if (rc == CYC_OK && s->win == 0 && s->maxc >= 2 && env_i64("CYC_SERIAL_ACC", 0) == 0) {
    // default-priority stream and timing-free events for the overlapped accumulation
    bool ok = hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking) == hipSuccess;
    for (int h = 0; h < 2 && ok; ++h)
      ok = hipEventCreateWithFlags(&s->ev_part[h], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&s->ev_acc[h], hipEventDisableTiming) == hipSuccess;
    if (ok) {
      s->maxc_half = s->maxc / 2;
    } else {
      (void)hipGetLastError();
      rc = CYC_ENOMEM;
    }
  }
  delete[] ar;
  if (rc != CYC_OK) {
    (void)hipGetLastError();
    free_state(s);
    return rc;
  }
  *out = s;
  return CYC_OK;
}

int cyc_create(cyc_state** out, const double* alphas_host, int32_t n_alpha, int32_t n_lag,
               uint32_t flags, void* stream) {
  return create_state(out, alphas_host, n_alpha, 0, n_lag, flags, false, 0, 0, stream);
}

int cyc_create_window(cyc_state** out, const double* alphas_host, int32_t n_alpha, int32_t n_lag, int32_t hop,
                      int32_t n_hops, uint32_t flags, void* stream) {
  if (n_hops < 1) return CYC_EINVAL;
  return create_state(out, alphas_host, n_alpha, 0, n_lag, flags, false, hop, n_hops, stream);
}

int cyc_create2(cyc_state** out, const double* alphas_host, int32_t n_alpha, int64_t lag_min, int32_t n_lag,
                uint32_t flags, void* stream) {
  return create_state(out, alphas_host, n_alpha, lag_min, n_lag, flags, true, 0, 0, stream);
}

}  // extern "C"

namespace {

// The virtual sample array of one input for a push: its pending samples (from
// absolute index nc + d) followed by the part of the new block from that index
// on.  n_pend / skip: pending count and leading samples of the block not needed.
VSrc input_src(const cyc_state* s, float2* const* bufs, int64_t d, const float2* blk, int64_t n, int64_t* n_pend,
               int64_t* skip) {
  *n_pend = std::max<int64_t>(0, s->L - (s->nc + d));
  *skip = std::min<int64_t>(n, std::max<int64_t>(0, s->nc + d - s->L));
  VSrc v;
  v.pend = bufs[s->cur];
  v.xin = blk + *skip;
  v.n_pend = *n_pend;
  v.n_avail = *n_pend + (n - *skip);
  return v;
}

// Keeps one input's samples from absolute index nc_new + d on for the next push.
hipError_t keep_input(const cyc_state* s, float2* const* bufs, const VSrc& v, int64_t n_pend, int64_t skip,
                      int64_t d, int64_t n, int64_t shift, int64_t L_new, hipStream_t st) {
  if (shift == 0) {
    // no chunk committed: append the new samples behind the pending ones
    const int64_t add = n - skip;
    if (add <= 0) return hipSuccess;
    VSrc a;
    a.pend = v.xin;
    a.xin = nullptr;
    a.n_pend = add;
    a.n_avail = add;
    return launch_vcopy(a, 0, add, bufs[s->cur] + n_pend, st);
  }
  const int64_t cnt = std::max<int64_t>(0, L_new - (s->nc + shift + d));
  return cnt > 0 ? launch_vcopy(v, shift, cnt, bufs[s->cur ^ 1], st) : hipSuccess;
}

bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

// Orders `st` after every accumulation issued on the side stream (the side
// stream is in order, so the last one covers them all).
hipError_t join_side(cyc_state* s, hipStream_t st) {
  if (!s->side || s->last_half < 0) return hipSuccess;
  return hipStreamWaitEvent(st, s->ev_acc[s->last_half], 0);
}

// Push of n samples of the leading input x and the trailing input y (y == x
// for one-input states).  Products n (absolute) pair x[n + dx + t] with
// y[n + dy] and are committed in chunks aligned to [c Kc, (c + 1) Kc); the
// chunk phase is referenced to y's index n + dy.  While fewer than G products
// are pending the push only appends its samples (unless `flush`, which
// commits every complete chunk; n may then be 0 with x = y = NULL).
int push_xy(cyc_state* s, const float2* x, const float2* y, int64_t n, hipStream_t st, bool flush = false) {
  const int64_t L_new = s->L + n;
  const int64_t n_used_new = std::max<int64_t>(0, L_new - (s->T - 1) - s->lagabs);
  const bool cap = capturing(st);
  const bool defer = !flush && !cap && s->G > 0 && n_used_new - s->nc < s->G;
  const int64_t chunks_new = defer ? 0 : n_used_new / s->Kc - s->nc / s->Kc;
  int64_t px = 0, sx = 0, py = 0, sy = 0;
  const VSrc vx = input_src(s, s->pend, s->dx, x, n, &px, &sx);
  const VSrc vy = s->two ? input_src(s, s->pendy, s->dy, y, n, &py, &sy) : vx;

  const bool overlap = s->side && chunks_new > 0 && !cap;
  if (!overlap && chunks_new > 0 && join_side(s, st) != hipSuccess) return fail_device(s);
  for (int64_t done = 0; overlap && done < chunks_new;) {
    // contraction into one workspace half here, its accumulation on the side stream
    const int h = s->half;
    const int nch = (int)std::min<int64_t>(s->maxc_half, chunks_new - done);
    const int64_t abs0 = s->nc + done * s->Kc;
    const int64_t TA2 = 2 * (int64_t)s->T * s->A;
    float2* part = s->part + (int64_t)h * s->maxc_half * TA2;
    double2* E = s->E + (int64_t)h * s->maxc_half * s->A;
    if ((s->acc_used[h] && hipStreamWaitEvent(st, s->ev_acc[h], 0) != hipSuccess) ||
        run_contract(s, vx, vy, done * s->Kc, (int64_t)nch * s->Kc, nch, st, part) != hipSuccess ||
        hipEventRecord(s->ev_part[h], st) != hipSuccess ||
        hipStreamWaitEvent(s->side, s->ev_part[h], 0) != hipSuccess ||
        launch_phase(s->alpha_r, s->A, abs0 + s->dy, s->Kc, nch, E, s->side) != hipSuccess ||
        launch_accumulate(s->S, part, E, s->T, s->A, nch, abs0 == 0 ? 1 : 0, s->tbl, s->side) != hipSuccess ||
        hipEventRecord(s->ev_acc[h], s->side) != hipSuccess)
      return fail_device(s);
    s->acc_used[h] = true;
    s->last_half = h;
    s->half ^= 1;
    done += nch;
  }
  for (int64_t done = 0; !overlap && done < chunks_new;) {
    const int nch = (int)std::min<int64_t>(s->maxc, chunks_new - done);
    const int64_t abs0 = s->nc + done * s->Kc;
    if (launch_phase(s->alpha_r, s->A, abs0 + s->dy, s->Kc, nch, s->E, st) != hipSuccess ||
        run_contract(s, vx, vy, done * s->Kc, (int64_t)nch * s->Kc, nch, st) != hipSuccess ||
        (s->win > 0 ? launch_window_store(s->ring, s->part, s->E, s->T, s->A, nch, abs0 / s->Kc, s->win, st)
                    : launch_accumulate(s->S, s->part, s->E, s->T, s->A, nch, abs0 == 0 ? 1 : 0, s->tbl, st)) !=
          hipSuccess)
      return fail_device(s);
    done += nch;
  }

  const int64_t shift = chunks_new * s->Kc;
  if (keep_input(s, s->pend, vx, px, sx, s->dx, n, shift, L_new, st) != hipSuccess ||
      (s->two && keep_input(s, s->pendy, vy, py, sy, s->dy, n, shift, L_new, st) != hipSuccess))
    return fail_device(s);
  if (shift > 0) s->cur ^= 1;
  s->L = L_new;
  s->nc += shift;
  return CYC_OK;
}

}  // namespace

extern "C" {

int cyc_push(cyc_state* s, const void* d_x, int64_t n, void* stream) {
  if (!s || n < 0 || (n > 0 && !d_x)) return CYC_EINVAL;
  if (s->poisoned) return CYC_ESTATE;
  if (n == 0) return CYC_OK;
  const float2* x = reinterpret_cast<const float2*>(d_x);
  return push_xy(s, x, x, n, as_stream(stream));
}

int cyc_push2(cyc_state* s, const void* d_x, const void* d_y, int64_t n, void* stream) {
  if (!s || n < 0 || (n > 0 && (!d_x || !d_y)) || !s->two) return CYC_EINVAL;
  if (s->poisoned) return CYC_ESTATE;
  if (n == 0) return CYC_OK;
  return push_xy(s, reinterpret_cast<const float2*>(d_x), reinterpret_cast<const float2*>(d_y), n,
                 as_stream(stream));
}

int cyc_read(cyc_state* s, void* d_R, void* d_Rc, int64_t* n_used, void* stream) {
  if (!s) return CYC_EINVAL;
  if (s->poisoned) return CYC_ESTATE;
  if ((s->tbl == 1 && d_Rc) || (s->tbl == 2 && d_R)) return CYC_EINVAL;  // a table the state does not keep
  hipStream_t st = as_stream(stream);
  const int c128 = (s->flags & CYC_OUT_C128) ? 1 : 0;
  const int64_t tbytes = (int64_t)s->T * s->A * (c128 ? 16 : 8);
  if (s->win > 0) {
    // the last min(win, hops committed) complete hops, phase from the window's first product
    const int64_t hops = s->nc / s->Kc;
    const int Wn = (int)std::min<int64_t>(s->win, hops);
    const int64_t nw = (int64_t)Wn * s->Kc;
    if (n_used) *n_used = nw;
    if (!d_R && !d_Rc) return CYC_OK;
    if (Wn == 0) {
      if ((d_R && launch_zero(d_R, tbytes, st) != hipSuccess) ||
          (d_Rc && launch_zero(d_Rc, tbytes, st) != hipSuccess))
        return fail_device(s);
      return CYC_OK;
    }
    const int64_t first = hops - Wn;
    if (launch_window_finalize(s->ring, s->win, (int)(first % s->win), Wn, s->T, s->A, s->alpha_r,
                               first * s->Kc + s->dy, nw, d_R, d_Rc, c128, st) != hipSuccess)
      return fail_device(s);
    return CYC_OK;
  }
  const int64_t nu = std::max<int64_t>(0, s->L - (s->T - 1) - s->lagabs);
  if (n_used) *n_used = nu;
  if (!d_R && !d_Rc) return CYC_OK;
  if (nu == 0) {
    if ((d_R && launch_zero(d_R, tbytes, st) != hipSuccess) ||
        (d_Rc && launch_zero(d_Rc, tbytes, st) != hipSuccess))
      return fail_device(s);
    return CYC_OK;
  }
  if (nu - s->nc >= s->Kc) {
    // complete chunks that coalescing pushes left pending
    const int rc = push_xy(s, nullptr, nullptr, 0, st, true);
    if (rc != CYC_OK) return rc;
  }
  if (join_side(s, st) != hipSuccess) return fail_device(s);
  const int64_t m = nu - s->nc;  // products of the pending partial chunk, < Kc
  if (m > 0) {
    VSrc vx;
    vx.pend = s->pend[s->cur];
    vx.xin = nullptr;
    vx.n_pend = s->L - s->nc - s->dx;
    vx.n_avail = vx.n_pend;
    VSrc vy = vx;
    if (s->two) {
      vy.pend = s->pendy[s->cur];
      vy.n_pend = s->L - s->nc - s->dy;
      vy.n_avail = vy.n_pend;
    }
    if (launch_phase(s->alpha_r, s->A, s->nc + s->dy, s->Kc, 1, s->E, st) != hipSuccess ||
        run_contract(s, vx, vy, 0, m, 1, st) != hipSuccess)
      return fail_device(s);
  }
  if (launch_finalize(s->S, s->nc > 0 ? 1 : 0, s->part, s->E, m > 0 ? 1 : 0, s->T, s->A, nu, d_R,
                      d_Rc, c128, st) != hipSuccess)
    return fail_device(s);
  return CYC_OK;
}

int cyc_reset(cyc_state* s) {
  if (!s) return CYC_EINVAL;
  s->L = 0;
  s->nc = 0;
  s->cur = 0;
  s->poisoned = false;
  return CYC_OK;
}

void cyc_destroy(cyc_state* s) {
  if (!s) return;
  (void)hipDeviceSynchronize();
  free_state(s);
}

int cyc_profile(cyc_state* s, int32_t enable) {
  if (!s) return CYC_EINVAL;
  s->prof = enable != 0;
  if (s->prof) {
    s->ev_used = 0;
    s->prof_work = 0.0;
  }
  return CYC_OK;
}

int cyc_profile_read(cyc_state* s, double* total_ms, int64_t* launches, double* work) {
  if (!s) return CYC_EINVAL;
  double ms = 0.0;
  for (size_t i = 0; i + 1 < s->ev_used; i += 2) {
    float t = 0.f;
    if (hipEventSynchronize(s->ev[i + 1]) != hipSuccess ||
        hipEventElapsedTime(&t, s->ev[i], s->ev[i + 1]) != hipSuccess)
      return CYC_EDEVICE;
    ms += t;
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = (int64_t)(s->ev_used / 2);
  if (work) *work = s->prof_work;
  return CYC_OK;
}

int cyc_kernel_cfg_count(void) {
  int n = 0;
  kernel_cfgs(&n);
  return n;
}

int cyc_kernel_cfg_info(int32_t idx, uint32_t* flags, int32_t* lag_tile, int32_t* alpha_tile,
                        int32_t* threads, const char** name) {
  int n = 0;
  const KernelCfg* c = kernel_cfgs(&n);
  if (idx < 0 || idx >= n) return CYC_EINVAL;
  if (flags)
    *flags = (uint32_t)c[idx].prec | (c[idx].split ? CYC_TW_SPLIT : 0u) |
             (c[idx].tbl == 1 ? CYC_TBL_R : 0u) | (c[idx].tbl == 2 ? CYC_TBL_RCONJ : 0u);
  if (lag_tile) *lag_tile = c[idx].tw;
  if (alpha_tile) *alpha_tile = c[idx].aw;
  if (threads) *threads = c[idx].nthreads;
  if (name) *name = c[idx].name;
  return CYC_OK;
}

int cyc_set_kernel_cfg(cyc_state* s, int32_t idx) {
  int n = 0;
  const KernelCfg* c = kernel_cfgs(&n);
  if (!s || idx < 0 || idx >= n) return CYC_EINVAL;
  const KernelCfg& cur = c[s->cfg];
  if (c[idx].prec != cur.prec || c[idx].split != cur.split || c[idx].ks != cur.ks || c[idx].tbl != cur.tbl)
    return CYC_EUNSUPPORTED;
  s->cfg = idx;
  return CYC_OK;
}

int cyc_autotune(int32_t n_alpha, int32_t n_lag, uint32_t flags, int32_t* best_cfg, double* best_ms,
                 void* stream) {
  if (n_alpha < 1 || n_lag < 1 || n_lag > kMaxLag) return CYC_EINVAL;
  hipStream_t st = as_stream(stream);
  // synthetic alphas (uniform grid) and samples (a fixed non-trivial pattern)
  std::vector<double> al(n_alpha);
  for (int i = 0; i < n_alpha; ++i) al[i] = -0.5 + (double)i / n_alpha;
  cyc_state* s = nullptr;
  int rc = cyc_create(&s, al.data(), n_alpha, n_lag, flags & ~CYC_OUT_C128, stream);
  if (rc != CYC_OK) return rc;
  s->G = 0;  // every timed push commits its 16 chunks
  const int64_t nsamp = (int64_t)s->Kc * 16 + n_lag - 1;
  float2* x = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&x), sizeof(float2) * nsamp) != hipSuccess) {
    cyc_destroy(s);
    return CYC_ENOMEM;
  }
  rc = CYC_OK;
  if (launch_pattern(x, nsamp, st) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess)
    rc = CYC_EDEVICE;
  int n = 0;
  const KernelCfg* c = kernel_cfgs(&n);
  const int prec = (int)(flags & CYC_OP_MASK), split = (flags & CYC_TW_SPLIT) ? 1 : 0;
  const int tbl = s->tbl;
  std::vector<int> cand;
  for (int i = 0; i < n; ++i)
    if (c[i].prec == prec && c[i].split == split && cyc_set_kernel_cfg(s, i) == CYC_OK) cand.push_back(i);
  // One timed push of 16 chunks (after a reset) on configuration i; < 0 on failure.
  auto timed_push = [&](int i) -> double {
    float t = 0.f;
    if (cyc_set_kernel_cfg(s, i) != CYC_OK) return -1.0;
    cyc_reset(s);
    if (hipEventRecord(e0, st) != hipSuccess || cyc_push(s, x, nsamp, stream) != CYC_OK ||
        hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&t, e0, e1) != hipSuccess)
      return -1.0;
    return (double)t;
  };
  // Warm the device up first, then time the candidates round-robin (three
  // rounds of one untimed and two timed pushes each) and take each one's
  // median: clock changes while tuning then affect every candidate alike.
  for (int w = 0; w < 10 && rc == CYC_OK && !cand.empty(); ++w)
    if (timed_push(cand[0]) < 0) rc = CYC_EDEVICE;
  std::vector<std::vector<double>> ts(cand.size());
  for (int round = 0; round < 3 && rc == CYC_OK; ++round)
    for (size_t k = 0; k < cand.size() && rc == CYC_OK; ++k)
      for (int rep = 0; rep < 3; ++rep) {
        const double t = timed_push(cand[k]);
        if (t < 0) {
          rc = CYC_EDEVICE;
          break;
        }
        if (rep > 0) ts[k].push_back(t);
      }
  int best = -1;
  double bms = 1e300;
  for (size_t k = 0; k < cand.size() && rc == CYC_OK; ++k) {
    std::sort(ts[k].begin(), ts[k].end());
    const double med = ts[k][ts[k].size() / 2];
    if (med < bms) {
      bms = med;
      best = cand[k];
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(x);
  cyc_destroy(s);
  if (rc != CYC_OK) return rc;
  if (best < 0) return CYC_EUNSUPPORTED;
  tune_store(TuneKey(device_arch(), prec, split + 2 * tbl, n_lag, a_bucket(n_alpha)), c[best].name);
  if (best_cfg) *best_cfg = best;
  if (best_ms) *best_ms = bms;
  return CYC_OK;
}

int cyc_query(const cyc_state* s, int64_t* n_pushed, int64_t* n_committed, int32_t* chunk,
              int32_t* kernel_cfg) {
  if (!s) return CYC_EINVAL;
  if (n_pushed) *n_pushed = s->L;
  if (n_committed) *n_committed = s->nc;
  if (chunk) *chunk = s->Kc;
  if (kernel_cfg) *kernel_cfg = s->cfg;
  return CYC_OK;
}

}  // extern "C"
