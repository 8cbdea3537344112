// Batches of stream states (cyc_batch_* in include/cyclo.h).
//
// Every stream keeps the single-state layout (reduced alphas, twiddle tables,
// FP64 accumulators, ping-pong pending buffers), packed into shared device
// arrays.  A push is split into rounds that fit the partial-sum workspace; a
// round is described by device-resident tables (jobs = one chunk of one
// stream, contraction work items, accumulation and pending-copy descriptors
// with their 256-element tiles) and executed by
//   reset counter -> batched phases -> persistent contraction ->
//   batched accumulation -> batched pending copies,
// captured once in a HIP graph and replayed after the tables are uploaded.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/cyclo.h"
#include "cyclo_internal.h"

using namespace cyclo;

int cyc_pick_cfg(int prec, int split, int T, int A);

namespace {

int64_t env_i64b(const char* name, int64_t dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  char* end = nullptr;
  long long r = std::strtoll(v, &end, 10);
  return (end && *end == 0) ? (int64_t)r : dflt;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t cnt, jobs, items, acc, acc_tiles, copy, copy_tiles, fin, bytes;
};

}  // namespace

struct cyc_batch {
  int n = 0, T = 0;
  uint32_t flags = 0;
  int Kc = 0, KS = 0, nsteps = 0, cfg = -1;
  std::vector<int> A;
  std::vector<int64_t> aoff, soff;
  double* alpha_r = nullptr;
  float2* Lo = nullptr;
  float2* H = nullptr;
  double2* S = nullptr;
  float2* pend = nullptr;
  int64_t PC = 0;  // pending capacity per buffer
  std::vector<int> cur;
  std::vector<int64_t> L, nc;
  float2* part = nullptr;
  int64_t part_cap = 0;  // complex values
  double2* E = nullptr;
  int64_t E_cap = 0;
  int JMAX = 0, IMAX = 0, ATMAX = 0, CTMAX = 0;
  Layout lay{};
  unsigned char* meta = nullptr;
  unsigned char* stage[2] = {nullptr, nullptr};
  hipEvent_t staged[2] = {nullptr, nullptr};
  int sidx = 0;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool graph_tried = false;
  bool use_graph = true;  // CYC_NO_GRAPH at creation turns graph capture off
  int grid = 0;
  int rounds = 0, graphed = 0;
  bool poisoned = false;
  // profiling: HIP events around every persistent contraction launch
  bool prof = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  double prof_work = 0.0;

  float2* pend_buf(int s, int which) const { return pend + ((int64_t)s * 2 + which) * PC; }
  BCounts* d_cnt() const { return reinterpret_cast<BCounts*>(meta + lay.cnt); }
  BJob* d_jobs() const { return reinterpret_cast<BJob*>(meta + lay.jobs); }
  BItem* d_items() const { return reinterpret_cast<BItem*>(meta + lay.items); }
  BAcc* d_acc() const { return reinterpret_cast<BAcc*>(meta + lay.acc); }
  BTile* d_acc_tiles() const { return reinterpret_cast<BTile*>(meta + lay.acc_tiles); }
  BCopy* d_copy() const { return reinterpret_cast<BCopy*>(meta + lay.copy); }
  BTile* d_copy_tiles() const { return reinterpret_cast<BTile*>(meta + lay.copy_tiles); }
  BFin* d_fin() const { return reinterpret_cast<BFin*>(meta + lay.fin); }
};

namespace {

void batch_free(cyc_batch* b) {
  if (!b) return;
  for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (int i = 0; i < 2; ++i) {
    if (b->staged[i]) (void)hipEventDestroy(b->staged[i]);
    if (b->stage[i]) (void)hipHostFree(b->stage[i]);
  }
  (void)hipFree(b->meta);
  (void)hipFree(b->alpha_r);
  (void)hipFree(b->Lo);
  (void)hipFree(b->H);
  (void)hipFree(b->S);
  (void)hipFree(b->pend);
  (void)hipFree(b->part);
  (void)hipFree(b->E);
  delete b;
}

template <typename T>
hipError_t dalloc_b(T** p, size_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T));
}

// Host-side image of one round's tables.
struct Round {
  std::vector<BJob> jobs;
  std::vector<BItem> items;
  std::vector<BAcc> acc;
  std::vector<BTile> acc_tiles;
  std::vector<BCopy> copy;
  std::vector<BTile> copy_tiles;
  std::vector<BFin> fin;
  int64_t part_used = 0, E_used = 0;
  void clear() {
    jobs.clear();
    items.clear();
    acc.clear();
    acc_tiles.clear();
    copy.clear();
    copy_tiles.clear();
    fin.clear();
    part_used = E_used = 0;
  }
};

void add_tiles(std::vector<BTile>& t, int desc, int64_t n) {
  for (int64_t off = 0; off < n; off += 256) {
    BTile x;
    x.desc = desc;
    x.pad = 0;
    x.off = off;
    t.push_back(x);
  }
}

// Uploads the round's tables (through a pinned staging buffer) on `st`.
hipError_t upload(cyc_batch* b, const Round& r, hipStream_t st) {
  const int si = b->sidx;
  b->sidx ^= 1;
  hipError_t e = hipEventSynchronize(b->staged[si]);  // staging buffer free again
  if (e != hipSuccess) return e;
  unsigned char* h = b->stage[si];
  BCounts c;
  std::memset(&c, 0, sizeof(c));
  c.n_jobs = (int)r.jobs.size();
  c.n_items = (int)r.items.size();
  c.n_acc_tiles = (int)r.acc_tiles.size();
  c.n_copy_tiles = (int)r.copy_tiles.size();
  c.n_fin_tiles = (int)r.acc_tiles.size();
  struct Sec {
    size_t off;
    const void* src;
    size_t bytes;
  } secs[] = {
      {b->lay.cnt, &c, sizeof(c)},
      {b->lay.jobs, r.jobs.data(), r.jobs.size() * sizeof(BJob)},
      {b->lay.items, r.items.data(), r.items.size() * sizeof(BItem)},
      {b->lay.acc, r.acc.data(), r.acc.size() * sizeof(BAcc)},
      {b->lay.acc_tiles, r.acc_tiles.data(), r.acc_tiles.size() * sizeof(BTile)},
      {b->lay.copy, r.copy.data(), r.copy.size() * sizeof(BCopy)},
      {b->lay.copy_tiles, r.copy_tiles.data(), r.copy_tiles.size() * sizeof(BTile)},
      {b->lay.fin, r.fin.data(), r.fin.size() * sizeof(BFin)},
  };
  for (const Sec& s : secs) {
    if (s.bytes == 0) continue;
    std::memcpy(h + s.off, s.src, s.bytes);
    e = hipMemcpyAsync(b->meta + s.off, h + s.off, s.bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
  }
  return hipEventRecord(b->staged[si], st);
}

BatchArgs batch_args(cyc_batch* b) {
  BatchArgs a;
  a.jobs = b->d_jobs();
  a.items = b->d_items();
  a.n_items = &b->d_cnt()->n_items;
  a.counter = &b->d_cnt()->counter;
  a.T = b->T;
  a.Kc = b->Kc;
  a.hs = (int)b->aoff.back();
  return a;
}

// Enqueues the push pipeline of one round on st.
// The persistent contraction launch, bracketed by HIP events while profiling
// (work = the round's products times lags times cycle frequencies).
hipError_t contract_launch(cyc_batch* b, double work, hipStream_t st) {
  int ncfg = 0;
  const KernelCfg& cfg = kernel_cfgs(&ncfg)[b->cfg];
  if (!b->prof) return cfg.blaunch(batch_args(b), b->grid, st);
  while (b->ev.size() < b->ev_used + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return hipErrorOutOfMemory;
    b->ev.push_back(e);
  }
  hipEvent_t e0 = b->ev[b->ev_used], e1 = b->ev[b->ev_used + 1];
  b->ev_used += 2;
  b->prof_work += work;
  hipError_t e = hipEventRecord(e0, st);
  if (e == hipSuccess) e = cfg.blaunch(batch_args(b), b->grid, st);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  return e;
}

double round_work(const cyc_batch* b, const std::vector<BJob>& jobs) {
  double w = 0.0;
  for (const BJob& j : jobs) w += (double)j.n_prod * j.A * b->T;
  return w;
}

hipError_t enqueue_push(cyc_batch* b, hipStream_t st, double work = 0.0) {
  hipError_t e = launch_batch_small(b->d_jobs(), b->d_cnt(), b->d_acc(), b->d_acc_tiles(),
                                    b->d_copy(), b->d_copy_tiles(), &b->d_cnt()->counter, 0, st);
  if (e != hipSuccess) return e;
  e = contract_launch(b, work, st);
  if (e != hipSuccess) return e;
  return launch_batch_small(b->d_jobs(), b->d_cnt(), b->d_acc(), b->d_acc_tiles(), b->d_copy(),
                            b->d_copy_tiles(), &b->d_cnt()->counter, 1, st);
}

// Captures the push pipeline once; falls back to direct launches if capture fails.
void ensure_graph(cyc_batch* b) {
  if (b->graph_tried) return;
  b->graph_tried = true;
  if (!b->use_graph) return;
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    b->cap = nullptr;
    return;
  }
  if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return;
  const hipError_t e = enqueue_push(b, b->cap);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(b->cap, &g);
  if (e != hipSuccess || e2 != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return;
  }
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    b->exec = nullptr;
    (void)hipGetLastError();
  }
}

hipError_t run_round(cyc_batch* b, const Round& r, hipStream_t st) {
  hipError_t e = upload(b, r, st);
  if (e != hipSuccess) return e;
  ++b->rounds;
  if (b->prof) {  // direct launches, so that the contraction can be timed
    b->graphed = 0;
    return enqueue_push(b, st, round_work(b, r.jobs));
  }
  ensure_graph(b);
  if (b->exec) {
    b->graphed = 1;
    return hipGraphLaunch(b->exec, st);
  }
  b->graphed = 0;
  return enqueue_push(b, st);
}

int items_per_job(const cyc_batch* b, int A) {
  int ncfg = 0;
  const KernelCfg& cfg = kernel_cfgs(&ncfg)[b->cfg];
  return ((b->T + cfg.tw - 1) / cfg.tw) * ((A + cfg.aw - 1) / cfg.aw);
}

void add_items(const cyc_batch* b, Round& r, int job, int A) {
  int ncfg = 0;
  const KernelCfg& cfg = kernel_cfgs(&ncfg)[b->cfg];
  const int ntt = (b->T + cfg.tw - 1) / cfg.tw, nat = (A + cfg.aw - 1) / cfg.aw;
  for (int tt = 0; tt < ntt; ++tt)
    for (int at = 0; at < nat; ++at) {
      BItem it;
      it.job = job;
      it.tt = tt;
      it.at = at;
      it.pad = 0;
      r.items.push_back(it);
    }
}

}  // namespace

extern "C" {

int cyc_batch_create(cyc_batch** out, int32_t n_streams, const int64_t* alpha_offsets,
                     const double* alphas, int32_t n_lag, uint32_t flags, void* stream) {
  if (!out || n_streams < 1 || !alpha_offsets || !alphas || n_lag < 1 || n_lag > 4096)
    return CYC_EINVAL;
  if (flags & (CYC_TBL_R | CYC_TBL_RCONJ)) return CYC_EUNSUPPORTED;  // batches keep both tables
  if (flags & ~(CYC_OP_MASK | CYC_TW_SPLIT | CYC_OUT_C128)) return CYC_EINVAL;
  const int prec = (int)(flags & CYC_OP_MASK);
  if (prec == 3) return CYC_EINVAL;
  const int split = (flags & CYC_TW_SPLIT) ? 1 : 0;
  if (split && prec == PREC_F32) return CYC_EUNSUPPORTED;
  if (alpha_offsets[0] != 0) return CYC_EINVAL;
  for (int s = 0; s < n_streams; ++s)
    if (alpha_offsets[s + 1] - alpha_offsets[s] < 1 ||
        alpha_offsets[s + 1] - alpha_offsets[s] > (1 << 24))
      return CYC_EINVAL;
  const int64_t atot = alpha_offsets[n_streams];
  for (int64_t i = 0; i < atot; ++i)
    if (!std::isfinite(alphas[i])) return CYC_EINVAL;

  cyc_batch* b = new (std::nothrow) cyc_batch();
  if (!b) return CYC_ENOMEM;
  b->n = n_streams;
  b->T = n_lag;
  b->flags = flags;
  b->use_graph = env_i64b("CYC_NO_GRAPH", 0) == 0;
  int amax = 1;
  b->A.resize(n_streams);
  b->aoff.assign(alpha_offsets, alpha_offsets + n_streams + 1);
  for (int s = 0; s < n_streams; ++s) {
    b->A[s] = (int)(alpha_offsets[s + 1] - alpha_offsets[s]);
    amax = std::max(amax, b->A[s]);
  }
  b->cfg = cyc_pick_cfg(prec, split, n_lag, amax);
  int ncfg = 0;
  const KernelCfg* cfgs = kernel_cfgs(&ncfg);
  if (b->cfg >= 0 && !cfgs[b->cfg].blaunch) {
    // tuned or forced choice has no batched form: default one of the mode
    b->cfg = -1;
    for (int i = 0; i < ncfg && b->cfg < 0; ++i)
      if (cfgs[i].prec == prec && cfgs[i].split == split && cfgs[i].blaunch &&
          cfgs[i].tw == (n_lag > 64 ? 128 : (n_lag > 32 ? 64 : 32)))
        b->cfg = i;
  }
  if (b->cfg < 0) {
    delete b;
    return CYC_EUNSUPPORTED;
  }
  const KernelCfg& cfg = cfgs[b->cfg];
  b->KS = cfg.ks;
  // Batches have parallelism across streams, so 16-bit operands use longer
  // chunks (fewer partial sums to write and fold); FP32 keeps 4096 products
  // per FP32-accumulated chunk for its accuracy budget.
  int64_t kc = env_i64b("CYC_CHUNK", prec == PREC_F32 ? 4096 : 16384);
  kc = std::max<int64_t>(cfg.ks, std::min<int64_t>(kc, 1 << 20));
  kc = (kc / cfg.ks) * cfg.ks;
  b->Kc = (int)kc;
  b->nsteps = b->Kc / b->KS;
  b->PC = (int64_t)b->Kc + b->T;
  b->soff.resize(n_streams + 1);
  b->soff[0] = 0;
  int64_t at = 0, ct = 0;
  for (int s = 0; s < n_streams; ++s) {
    const int64_t n2 = 2 * (int64_t)b->T * b->A[s];
    b->soff[s + 1] = b->soff[s] + n2;
    at += (n2 + 255) / 256;
    ct += (b->PC + 255) / 256;
  }
  b->ATMAX = (int)at;
  b->CTMAX = (int)ct;
  // 4 GiB holds one push of the 512-stream benchmark mix in a single round
  // (1 GiB needed four: BF16 5.2-5.4e13 against 5.5e13 (alpha,tau)*samples/s)
  const int64_t ws_bytes = env_i64b("CYC_WORKSPACE_MB", 4096) << 20;
  b->part_cap = std::max<int64_t>(2 * (int64_t)b->T * amax, ws_bytes / 8);
  b->E_cap = std::max<int64_t>(amax, b->part_cap / (2 * (int64_t)b->T));
  b->JMAX = 32768;
  b->IMAX = 1 << 20;
  Layout& l = b->lay;
  size_t o = 0;
  l.cnt = o;
  o = align256(o + sizeof(BCounts));
  l.jobs = o;
  o = align256(o + (size_t)std::max(b->JMAX, n_streams) * sizeof(BJob));
  l.items = o;
  o = align256(o + (size_t)b->IMAX * sizeof(BItem));
  l.acc = o;
  o = align256(o + (size_t)n_streams * sizeof(BAcc));
  l.acc_tiles = o;
  o = align256(o + (size_t)b->ATMAX * sizeof(BTile));
  l.copy = o;
  o = align256(o + (size_t)n_streams * sizeof(BCopy));
  l.copy_tiles = o;
  o = align256(o + (size_t)b->CTMAX * sizeof(BTile));
  l.fin = o;
  o = align256(o + (size_t)n_streams * sizeof(BFin));
  l.bytes = o;

  b->cur.assign(n_streams, 0);
  b->L.assign(n_streams, 0);
  b->nc.assign(n_streams, 0);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::vector<double> ar(atot);
  for (int64_t i = 0; i < atot; ++i) ar[i] = alphas[i] - std::nearbyint(alphas[i]);
  int rc = CYC_OK;
  if (dalloc_b(&b->alpha_r, atot) != hipSuccess || dalloc_b(&b->Lo, atot * b->KS) != hipSuccess ||
      dalloc_b(&b->H, atot * b->nsteps) != hipSuccess ||
      dalloc_b(&b->S, b->soff[n_streams]) != hipSuccess ||
      dalloc_b(&b->pend, (size_t)n_streams * 2 * b->PC) != hipSuccess ||
      dalloc_b(&b->part, b->part_cap) != hipSuccess || dalloc_b(&b->E, b->E_cap) != hipSuccess ||
      dalloc_b(&b->meta, l.bytes) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&b->stage[0]), l.bytes, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&b->stage[1]), l.bytes, hipHostMallocDefault) != hipSuccess ||
      hipEventCreate(&b->staged[0]) != hipSuccess || hipEventCreate(&b->staged[1]) != hipSuccess)
    rc = CYC_ENOMEM;
  if (rc == CYC_OK) {
    b->grid = cfg.bgrid ? cfg.bgrid() : 0;
    if (b->grid <= 0) rc = CYC_EDEVICE;
  }
  if (rc == CYC_OK &&
      (hipMemcpyAsync(b->alpha_r, ar.data(), sizeof(double) * atot, hipMemcpyHostToDevice, st) != hipSuccess ||
       launch_tables(b->alpha_r, (int)atot, b->KS, b->nsteps, b->Lo, b->H, st) != hipSuccess ||
       hipStreamSynchronize(st) != hipSuccess))
    rc = CYC_EDEVICE;
  if (rc != CYC_OK) {
    (void)hipGetLastError();
    batch_free(b);
    return rc;
  }
  *out = b;
  return CYC_OK;
}

int cyc_batch_push(cyc_batch* b, const void* const* d_x, const int64_t* n, void* stream) {
  if (!b || !d_x || !n) return CYC_EINVAL;
  for (int s = 0; s < b->n; ++s)
    if (n[s] < 0 || (n[s] > 0 && !d_x[s])) return CYC_EINVAL;
  if (b->poisoned) return CYC_ESTATE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  b->rounds = 0;

  std::vector<int64_t> chunks(b->n), n_pend(b->n);
  std::vector<VSrc> vs(b->n);
  for (int s = 0; s < b->n; ++s) {
    n_pend[s] = b->L[s] - b->nc[s];
    const int64_t Lnew = b->L[s] + n[s];
    const int64_t nu = std::max<int64_t>(0, Lnew - b->T + 1);
    chunks[s] = nu / b->Kc - b->nc[s] / b->Kc;
    vs[s].pend = b->pend_buf(s, b->cur[s]);
    vs[s].xin = reinterpret_cast<const float2*>(d_x[s]);
    vs[s].n_pend = n_pend[s];
    vs[s].n_avail = n_pend[s] + n[s];
  }

  Round r;
  int s_acc = -1;  // stream of the open accumulation descriptor
  auto close_acc = [&]() { s_acc = -1; };
  auto flush = [&](bool last) -> hipError_t {
    if (last) {
      for (int s = 0; s < b->n; ++s) {
        if (n[s] == 0) continue;
        const int64_t shift = chunks[s] * b->Kc;
        const int64_t npn = n_pend[s] + n[s] - shift;
        BCopy c;
        if (shift == 0) {
          c.v.pend = reinterpret_cast<const float2*>(d_x[s]);
          c.v.xin = nullptr;
          c.v.n_pend = n[s];
          c.v.n_avail = n[s];
          c.shift = 0;
          c.n = n[s];
          c.dst = b->pend_buf(s, b->cur[s]) + n_pend[s];
        } else {
          c.v = vs[s];
          c.shift = shift;
          c.n = npn;
          c.dst = b->pend_buf(s, b->cur[s] ^ 1);
        }
        add_tiles(r.copy_tiles, (int)r.copy.size(), c.n);
        r.copy.push_back(c);
      }
    }
    if (r.jobs.empty() && r.copy.empty()) return hipSuccess;
    for (size_t i = 0; i < r.acc.size(); ++i) add_tiles(r.acc_tiles, (int)i, r.acc[i].n2);
    const hipError_t e = run_round(b, r, st);
    r.clear();
    close_acc();
    return e;
  };

  for (int s = 0; s < b->n; ++s) {
    const int A = b->A[s];
    const int64_t per_part = 2 * (int64_t)b->T * A;
    const int ipj = items_per_job(b, A);
    for (int64_t c = 0; c < chunks[s]; ++c) {
      if ((int)r.jobs.size() + 1 > b->JMAX || (int64_t)r.items.size() + ipj > b->IMAX ||
          r.part_used + per_part > b->part_cap || r.E_used + A > b->E_cap) {
        if (flush(false) != hipSuccess) {
          b->poisoned = true;
          return CYC_EDEVICE;
        }
      }
      BJob j;
      j.v = vs[s];
      j.v_off = c * b->Kc;
      j.n_prod = b->Kc;
      j.abs_base = b->nc[s] + c * b->Kc;
      j.alpha_r = b->alpha_r + b->aoff[s];
      j.H = b->H + b->aoff[s];
      j.Lo = b->Lo + b->aoff[s] * b->KS;
      j.part = b->part + r.part_used;
      j.E = b->E + r.E_used;
      j.A = A;
      j.pad = 0;
      r.part_used += per_part;
      r.E_used += A;
      const int jid = (int)r.jobs.size();
      r.jobs.push_back(j);
      add_items(b, r, jid, A);
      if (s_acc != s) {
        BAcc a;
        a.S = b->S + b->soff[s];
        a.n2 = per_part;
        a.job0 = jid;
        a.njobs = 0;
        a.A = A;
        a.first = j.abs_base == 0 ? 1 : 0;
        r.acc.push_back(a);
        s_acc = s;
      }
      r.acc.back().njobs += 1;
    }
  }
  if (flush(true) != hipSuccess) {
    b->poisoned = true;
    return CYC_EDEVICE;
  }
  for (int s = 0; s < b->n; ++s) {
    if (n[s] == 0) continue;
    if (chunks[s] > 0) b->cur[s] ^= 1;
    b->L[s] += n[s];
    b->nc[s] += chunks[s] * b->Kc;
  }
  return CYC_OK;
}

int cyc_batch_read(cyc_batch* b, void* const* d_R, void* const* d_Rc, int64_t* n_used,
                   void* stream) {
  if (!b) return CYC_EINVAL;
  if (b->poisoned) return CYC_ESTATE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int c128 = (b->flags & CYC_OUT_C128) ? 1 : 0;
  if (n_used)
    for (int s = 0; s < b->n; ++s) n_used[s] = std::max<int64_t>(0, b->L[s] - b->T + 1);
  if (!d_R && !d_Rc) return CYC_OK;
  int ncfg = 0;
  const KernelCfg& cfg = kernel_cfgs(&ncfg)[b->cfg];
  Round r;
  auto flush = [&]() -> hipError_t {
    if (r.fin.empty()) return hipSuccess;
    for (size_t i = 0; i < r.fin.size(); ++i) add_tiles(r.acc_tiles, (int)i, 2 * r.fin[i].TA);
    hipError_t e = upload(b, r, st);
    if (e == hipSuccess)
      e = launch_batch_small(b->d_jobs(), b->d_cnt(), b->d_acc(), b->d_acc_tiles(), b->d_copy(),
                             b->d_copy_tiles(), &b->d_cnt()->counter, 0, st);
    if (e == hipSuccess && !r.jobs.empty()) e = contract_launch(b, round_work(b, r.jobs), st);
    if (e == hipSuccess) e = launch_batch_finalize(b->d_jobs(), b->d_fin(), b->d_acc_tiles(), b->d_cnt(), st);
    r.clear();
    return e;
  };
  for (int s = 0; s < b->n; ++s) {
    void* R = d_R ? d_R[s] : nullptr;
    void* Rc = d_Rc ? d_Rc[s] : nullptr;
    if (!R && !Rc) continue;
    const int A = b->A[s];
    const int64_t per_part = 2 * (int64_t)b->T * A;
    const int64_t nu = std::max<int64_t>(0, b->L[s] - b->T + 1);
    const int64_t m = nu - b->nc[s];
    const int ipj = m > 0 ? items_per_job(b, A) : 0;
    if ((int)r.jobs.size() + 1 > b->JMAX || (int64_t)r.items.size() + ipj > b->IMAX ||
        r.part_used + per_part > b->part_cap || r.E_used + A > b->E_cap) {
      if (flush() != hipSuccess) {
        b->poisoned = true;
        return CYC_EDEVICE;
      }
    }
    BFin f;
    f.S = b->S + b->soff[s];
    f.R = R;
    f.Rc = Rc;
    f.TA = (int64_t)b->T * A;
    f.nd = nu > 0 ? (double)nu : 1.0;
    f.job = -1;
    f.hasS = (nu > 0 && b->nc[s] > 0) ? 1 : 0;
    f.A = A;
    f.c128 = c128;
    if (nu > 0 && m > 0) {
      BJob j;
      j.v.pend = b->pend_buf(s, b->cur[s]);
      j.v.xin = nullptr;
      j.v.n_pend = b->L[s] - b->nc[s];
      j.v.n_avail = j.v.n_pend;
      j.v_off = 0;
      j.n_prod = m;
      j.abs_base = b->nc[s];
      j.alpha_r = b->alpha_r + b->aoff[s];
      j.H = b->H + b->aoff[s];
      j.Lo = b->Lo + b->aoff[s] * b->KS;
      j.part = b->part + r.part_used;
      j.E = b->E + r.E_used;
      j.A = A;
      j.pad = 0;
      r.part_used += per_part;
      r.E_used += A;
      f.job = (int)r.jobs.size();
      r.jobs.push_back(j);
      add_items(b, r, f.job, A);
    }
    r.fin.push_back(f);
  }
  if (flush() != hipSuccess) {
    b->poisoned = true;
    return CYC_EDEVICE;
  }
  return CYC_OK;
}

int cyc_batch_reset(cyc_batch* b) {
  if (!b) return CYC_EINVAL;
  std::fill(b->L.begin(), b->L.end(), 0);
  std::fill(b->nc.begin(), b->nc.end(), 0);
  std::fill(b->cur.begin(), b->cur.end(), 0);
  b->poisoned = false;
  return CYC_OK;
}

void cyc_batch_destroy(cyc_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  batch_free(b);
}

int cyc_batch_profile(cyc_batch* b, int32_t enable) {
  if (!b) return CYC_EINVAL;
  b->prof = enable != 0;
  if (b->prof) {
    b->ev_used = 0;
    b->prof_work = 0.0;
  }
  return CYC_OK;
}

int cyc_batch_profile_read(cyc_batch* b, double* total_ms, int64_t* launches, double* work) {
  if (!b) return CYC_EINVAL;
  double ms = 0.0;
  for (size_t i = 0; i + 1 < b->ev_used; i += 2) {
    float t = 0.f;
    if (hipEventSynchronize(b->ev[i + 1]) != hipSuccess ||
        hipEventElapsedTime(&t, b->ev[i], b->ev[i + 1]) != hipSuccess)
      return CYC_EDEVICE;
    ms += t;
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = (int64_t)(b->ev_used / 2);
  if (work) *work = b->prof_work;
  return CYC_OK;
}

int cyc_batch_query(const cyc_batch* b, int32_t* kernel_cfg, int32_t* rounds, int32_t* graph) {
  if (!b) return CYC_EINVAL;
  if (kernel_cfg) *kernel_cfg = b->cfg;
  if (rounds) *rounds = b->rounds;
  if (graph) *graph = b->graphed;
  return CYC_OK;
}

}  // extern "C"
