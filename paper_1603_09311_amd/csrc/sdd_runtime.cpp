// Host runtime behind the C ABI declared in include/sdd.h: context,
// workspace allocator (the caller's device buffer is the only device memory
// used), resident models, request preparation, batched persistent launches,
// the plain per-node form and the served (continuous-batching) loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sdd.h"
#include "sdd_device.h"

namespace sdd {
hipError_t launch_walk_plain(const DevReq *req_dev, uint32_t node, uint32_t p0, uint32_t count, uint64_t rec0,
                             hipStream_t st);
hipError_t launch_walk_persist(int precision, const DevReq *reqs_dev, uint32_t n_req,
                               const uint32_t *wave_start_dev, uint32_t blocks, uint32_t threads, hipStream_t st);
hipError_t launch_reduce(const NodeJob *jobs_dev, uint32_t n_jobs, hipStream_t st);
hipError_t launch_reset(uint32_t *tile_counters, unsigned long long *done, uint32_t n, hipStream_t st);
int persist_blocks_per_cu(int precision, uint32_t threads);
}  // namespace sdd

using namespace sdd;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static sdd_status fail(sdd_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(SDD_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// Workspace allocator: first fit over the caller's device buffer.
// ---------------------------------------------------------------------------
class Arena {
 public:
  void init(char *base, size_t bytes) {
    base_ = base;
    size_ = bytes;
    free_.clear();
    if (bytes) free_[0] = bytes;
    used_ = 0;
  }
  // Returns nullptr when no free block is large enough.
  char *alloc(size_t bytes) {
    bytes = round(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        live_[off] = bytes;
        used_ += bytes;
        return base_ + off;
      }
    }
    return nullptr;
  }
  void release(char *p) {
    if (!p) return;
    const size_t off = (size_t)(p - base_);
    auto it = live_.find(off);
    if (it == live_.end()) return;
    size_t len = it->second;
    live_.erase(it);
    used_ -= len;
    size_t start = off;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first == off + len) {
      len += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == start) {
        start = pv->first;
        len += pv->second;
        free_.erase(pv);
      }
    }
    free_[start] = len;
  }
  size_t largest_free() const {
    size_t m = 0;
    for (auto &kv : free_) m = std::max(m, kv.second);
    return m;
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }
  static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }

 private:
  char *base_ = nullptr;
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_, live_;
};

// ---------------------------------------------------------------------------
// Models and prepared requests
// ---------------------------------------------------------------------------
struct HostModel {
  sdd_model_desc desc;
  std::vector<sdd_region> regions;
  char *dev = nullptr;   // resident DevModel in the workspace
  std::atomic<int> in_flight{0};  // prepared requests referencing it
};

static constexpr uint32_t kPilotPaths = 4096;
static constexpr uint32_t kMaxTargetPaths = 1u << 20;
static constexpr uint32_t kDefaultMaxSteps = 2000000000u;

// One request's device allocations and bookkeeping for one pass (fixed
// paths, or the pilot / the extension of a target-SE request).
struct Prepared {
  ~Prepared();
  sdd_ctx *owner = nullptr;        // releases the model hold on destruction
  sdd_request req;                 // copy; pointers below are owned copies
  const HostModel *model = nullptr;
  std::vector<double> g, nodes;
  std::vector<uint32_t> pbeg, pcnt;  // this pass's path range per node
  std::vector<uint32_t> pbeg_all, pcnt_all;  // the request's full ranges
  DevReq dreq{};
  std::vector<DevTile> tiles;
  uint64_t n_paths = 0;            // paths in this pass
  std::vector<uint64_t> rec_off;   // per node record offset of this pass
  // device allocations
  char *d_g = nullptr, *d_nodes = nullptr, *d_tiles = nullptr, *d_recs = nullptr;
  char *d_recs_pilot = nullptr;    // pilot records kept for the final reduction
  std::vector<uint64_t> pilot_off; // per node pilot record offset
  std::vector<uint32_t> pilot_cnt;
  int pass = 0;                    // 0 fixed/pilot, 1 extension
};

struct Ticket {
  std::unique_ptr<Prepared> P;
  sdd_result res{};
  sdd_status status = SDD_OK;
  bool done = false, cancelled = false;
  std::string error;
};

struct sdd_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  Arena arena;
  int cus = 0;
  sdd_tuning tuning{256, 0, 512, 4096};
  std::mutex exec;                 // one launch sequence at a time on the stream
  std::mutex mu;                   // guards everything below and the arena
  char *alloc(size_t b) {
    std::lock_guard<std::mutex> lk(mu);
    return arena.alloc(b);
  }
  void release(char *p) {
    std::lock_guard<std::mutex> lk(mu);
    arena.release(p);
  }
  std::unordered_map<uint32_t, std::unique_ptr<HostModel>> models;
  uint32_t next_model = 1;
  // served mode
  std::unordered_map<uint64_t, std::shared_ptr<Ticket>> tickets;
  std::deque<std::shared_ptr<Ticket>> queue;
  uint64_t next_ticket = 1;
  std::condition_variable cv, done_cv;
  std::thread worker;
  bool stop = false;
  // timing of the last walk / reduction launches (guarded by exec)
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  sdd_stats stats{};
};

// Takes no lock: a Prepared may be destroyed while ctx->mu is held.
Prepared::~Prepared() {
  if (owner && model) const_cast<HostModel *>(model)->in_flight.fetch_sub(1);
}

static double alpha_of(const sdd_request &r, const HostModel &m, double sigma) {
  const double pi = 3.14159265358979323846264338327950288;
  if (r.freq_hz > 0.0) {
    const double omega = 2.0 * pi * r.freq_hz;
    const double mu0 = 4.0e-7 * pi;
    const double L = m.desc.length_unit_m;
    return omega * mu0 * sigma * (L * L);
  }
  return r.alpha_direct * sigma;
}

static sdd_status validate(sdd_ctx *ctx, const sdd_request *r, const HostModel **out_model) {
  if (!r) return fail(SDD_E_INVALID, "request is NULL");
  auto it = ctx->models.find(r->model);
  if (it == ctx->models.end()) return fail(SDD_E_NOTFOUND, "unknown model %u", r->model);
  const HostModel &m = *it->second;
  const sdd_model_desc &d = m.desc;
  if (r->precision != SDD_FP64 && r->precision != SDD_FP32_MIXED)
    return fail(SDD_E_INVALID, "precision must be SDD_FP64 or SDD_FP32_MIXED");
  if (!(r->dt > 0.0) || !std::isfinite(r->dt)) return fail(SDD_E_INVALID, "dt must be > 0 and finite");
  const double half = 0.5 * std::min(d.y_hi - d.y_lo, d.z_hi - d.z_lo);
  if (!(7.0 * std::sqrt(r->dt) < half))
    return fail(SDD_E_INVALID, "dt too large: 7 sqrt(dt) must stay below half the shorter side (%g)", half);
  if (r->g_samples < 2 || !r->g_tables) return fail(SDD_E_INVALID, "g_samples must be >= 2 with g_tables set");
  if (r->g_samples > (1u << 26)) return fail(SDD_E_INVALID, "g_samples too large");
  if (r->n_nodes && !r->nodes_yz) return fail(SDD_E_INVALID, "nodes_yz is NULL");
  if (r->stream >= 0x80000000u) return fail(SDD_E_INVALID, "stream must be < 2^31");
  if (r->freq_hz < 0.0 || !std::isfinite(r->freq_hz)) return fail(SDD_E_INVALID, "freq_hz must be >= 0");
  if (r->freq_hz == 0.0 && (!(r->alpha_direct >= 0.0) || !std::isfinite(r->alpha_direct)))
    return fail(SDD_E_INVALID, "alpha_direct must be >= 0 when freq_hz == 0");
  if (r->flags != 0) return fail(SDD_E_INVALID, "flags must be 0");
  if (!(r->target_rel_se >= 0.0) || !std::isfinite(r->target_rel_se))
    return fail(SDD_E_INVALID, "target_rel_se must be >= 0");
  for (uint32_t k = 0; k < 4 * 2 * r->g_samples; ++k)
    if (!std::isfinite(r->g_tables[k])) return fail(SDD_E_INVALID, "g_tables holds a non-finite value");
  for (uint32_t j = 0; j < r->n_nodes; ++j) {
    const double y = r->nodes_yz[2 * j], z = r->nodes_yz[2 * j + 1];
    if (!(y > d.y_lo && y < d.y_hi && z > d.z_lo && z < d.z_hi))
      return fail(SDD_E_INVALID, "node %u (%g, %g) is not strictly inside the domain", j, y, z);
    if (r->precision == SDD_FP32_MIXED) {
      const float fy = (float)y, fz = (float)z;
      if (!(fy > (float)d.y_lo && fy < (float)d.y_hi && fz > (float)d.z_lo && fz < (float)d.z_hi))
        return fail(SDD_E_INVALID, "node %u lies on a wall once rounded to FP32", j);
    }
    const uint64_t b = r->path_begin ? r->path_begin[j] : 0;
    const uint64_t c = r->path_count ? r->path_count[j] : r->paths_uniform;
    if (r->target_rel_se == 0.0) {
      if (c < 1) return fail(SDD_E_INVALID, "node %u has no paths", j);
      if (b + c > 0x100000000ull) return fail(SDD_E_INVALID, "node %u: path range beyond 2^32", j);
    } else if (b + kMaxTargetPaths > 0x100000000ull) {
      return fail(SDD_E_INVALID, "node %u: path range beyond 2^32", j);
    }
  }
  *out_model = &m;
  return SDD_OK;
}

static void fill_devreq(Prepared &P) {
  const sdd_request &r = P.req;
  const HostModel &m = *P.model;
  DevReq &q = P.dreq;
  std::memset(&q, 0, sizeof(q));
  q.y_lo = m.desc.y_lo; q.y_hi = m.desc.y_hi; q.z_lo = m.desc.z_lo; q.z_hi = m.desc.z_hi;
  q.dt = r.dt;
  q.s = std::sqrt(r.dt);
  q.thr = 22.9 * r.dt;
  // the FP32 walk measures positions from the centre of the domain
  q.ymid = 0.5 * (q.y_lo + q.y_hi);
  q.zmid = 0.5 * (q.z_lo + q.z_hi);
  const uint32_t np = (uint32_t)m.regions.size();
  q.nprims = np;
  for (uint32_t k = 0; k < np; ++k) {
    q.c[k] = alpha_of(r, m, m.regions[k].sigma) * r.dt / 2.0;
    q.kind[k] = m.regions[k].kind;
    const double *v = m.regions[k].v;
    for (int i = 0; i < 6; ++i) q.pd[k][i] = v[i];
    // centred FP32 geometry: y-coordinates minus ymid, z-coordinates minus zmid
    switch (m.regions[k].kind) {
      case SDD_HALF_Z_LT: q.pf[k][0] = (float)(v[0] - q.zmid); break;
      case SDD_HALF_Y_LT: q.pf[k][0] = (float)(v[0] - q.ymid); break;
      case SDD_BOX:
        q.pf[k][0] = (float)(v[0] - q.ymid); q.pf[k][1] = (float)(v[1] - q.ymid);
        q.pf[k][2] = (float)(v[2] - q.zmid); q.pf[k][3] = (float)(v[3] - q.zmid);
        break;
      default:
        for (int i = 0; i < 6; i += 2) {
          q.pf[k][i] = (float)(v[i] - q.ymid);
          q.pf[k][i + 1] = (float)(v[i + 1] - q.zmid);
        }
    }
  }
  q.c[np] = alpha_of(r, m, m.desc.sigma_background) * r.dt / 2.0;
  q.fhy = (float)(0.5 * (q.y_hi - q.y_lo));
  q.fhz = (float)(0.5 * (q.z_hi - q.z_lo));
  q.fs = (float)q.s;
  q.fdt = (float)q.dt;
  q.fthr = 22.9f * q.fdt;
  q.fscr = 0.5f * q.fthr;
  for (uint32_t k = 0; k <= np; ++k) q.fc[k] = (float)q.c[k];
  q.key0 = (uint32_t)(r.seed & 0xFFFFFFFFu);
  q.key1 = (uint32_t)(r.seed >> 32);
  q.ctr3 = 2u * r.stream;
  q.max_steps = r.max_steps ? r.max_steps : kDefaultMaxSteps;
  q.precision = (uint32_t)r.precision;
  q.M = r.g_samples - 1;
  q.model = reinterpret_cast<const DevModel *>(m.dev);
}

// Copy the request's inputs; set up the first pass's path ranges.
static sdd_status prepare(sdd_ctx *ctx, const sdd_request *r, std::unique_ptr<Prepared> &out) {
  const HostModel *m = nullptr;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    sdd_status st = validate(ctx, r, &m);
    if (st != SDD_OK) return st;
    const_cast<HostModel *>(m)->in_flight.fetch_add(1);   // the model outlives the request
  }
  auto P = std::make_unique<Prepared>();
  P->owner = ctx;
  P->req = *r;
  P->model = m;
  P->g.assign(r->g_tables, r->g_tables + (size_t)8 * r->g_samples);
  P->nodes.assign(r->nodes_yz, r->nodes_yz + (size_t)2 * r->n_nodes);
  const uint32_t n = r->n_nodes;
  P->pbeg_all.resize(n);
  P->pcnt_all.resize(n);
  for (uint32_t j = 0; j < n; ++j) {
    P->pbeg_all[j] = r->path_begin ? r->path_begin[j] : 0u;
    P->pcnt_all[j] = r->path_count ? r->path_count[j] : r->paths_uniform;
  }
  P->req.g_tables = nullptr;
  P->req.nodes_yz = nullptr;
  P->req.path_begin = nullptr;
  P->req.path_count = nullptr;
  P->pbeg = P->pbeg_all;
  P->pcnt = P->pcnt_all;
  if (r->target_rel_se > 0.0)
    for (uint32_t j = 0; j < n; ++j) P->pcnt[j] = kPilotPaths;
  fill_devreq(*P);
  out = std::move(P);
  return SDD_OK;
}

static void build_tiles(Prepared &P, uint32_t tile_paths) {
  const uint32_t n = (uint32_t)P.pbeg.size();
  P.tiles.clear();
  P.rec_off.assign(n + 1, 0);
  uint64_t off = 0;
  for (uint32_t j = 0; j < n; ++j) {
    P.rec_off[j] = off;
    const uint32_t b = P.pbeg[j], c = P.pcnt[j];
    for (uint32_t k = 0; k < c; k += tile_paths) {
      DevTile t{};
      t.node = j;
      t.p0 = b + k;
      t.count = std::min(tile_paths, c - k);
      t.rec0 = off + k;
      P.tiles.push_back(t);
    }
    off += c;
  }
  P.rec_off[n] = off;
  P.n_paths = off;
}

static size_t pass_bytes(const Prepared &P) {
  return Arena::round(P.g.size() * 8) + Arena::round(P.nodes.size() * 8 + 16) +
         Arena::round(P.tiles.size() * sizeof(DevTile) + 16) + Arena::round(P.n_paths * sizeof(PathRec) + 16);
}

static void release_pass(sdd_ctx *ctx, Prepared &P) {
  ctx->release(P.d_g);
  ctx->release(P.d_nodes);
  ctx->release(P.d_tiles);
  ctx->release(P.d_recs);
  P.d_g = P.d_nodes = P.d_tiles = P.d_recs = nullptr;
}

static void release_all(sdd_ctx *ctx, Prepared &P) {
  release_pass(ctx, P);
  ctx->release(P.d_recs_pilot);
  P.d_recs_pilot = nullptr;
}

// Allocate and upload one pass's inputs (caller holds ctx->mu).
static sdd_status upload_pass(sdd_ctx *ctx, Prepared &P) {
  build_tiles(P, ctx->tuning.tile_paths ? ctx->tuning.tile_paths : 512u);
  P.d_g = ctx->alloc(P.g.size() * 8);
  P.d_nodes = ctx->alloc(P.nodes.size() * 8 + 16);
  P.d_tiles = ctx->alloc(P.tiles.size() * sizeof(DevTile) + 16);
  P.d_recs = ctx->alloc(P.n_paths * sizeof(PathRec) + 16);
  if (!P.d_g || !P.d_nodes || !P.d_tiles || !P.d_recs) {
    release_pass(ctx, P);
    size_t largest;
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      largest = ctx->arena.largest_free();
    }
    return fail(SDD_E_NOMEM, "request needs %zu bytes of workspace; largest free block is %zu", pass_bytes(P),
                largest);
  }
  HIP_TRY(hipMemcpyAsync(P.d_g, P.g.data(), P.g.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  if (!P.nodes.empty())
    HIP_TRY(hipMemcpyAsync(P.d_nodes, P.nodes.data(), P.nodes.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  if (!P.tiles.empty())
    HIP_TRY(hipMemcpyAsync(P.d_tiles, P.tiles.data(), P.tiles.size() * sizeof(DevTile), hipMemcpyHostToDevice,
                           ctx->stream));
  P.dreq.g = reinterpret_cast<const double *>(P.d_g);
  P.dreq.nodes = reinterpret_cast<const double *>(P.d_nodes);
  P.dreq.tiles = reinterpret_cast<const DevTile *>(P.d_tiles);
  P.dreq.recs = reinterpret_cast<PathRec *>(P.d_recs);
  P.dreq.n_tiles = (uint32_t)P.tiles.size();
  return SDD_OK;
}

// ---------------------------------------------------------------------------
// One persistent launch over a set of passes (caller holds ctx->mu).
// ---------------------------------------------------------------------------
struct BatchScratch {
  char *d_reqs = nullptr, *d_ctr = nullptr, *d_done = nullptr, *d_ws = nullptr;
  void release(sdd_ctx *ctx) {
    ctx->release(d_reqs);
    ctx->release(d_ctr);
    ctx->release(d_done);
    ctx->release(d_ws);
    d_reqs = d_ctr = d_done = d_ws = nullptr;
  }
};

static void launch_shape(sdd_ctx *ctx, int precision, uint32_t &blocks, uint32_t &threads) {
  threads = ctx->tuning.block_threads ? ctx->tuning.block_threads : 256u;
  uint32_t per_cu = ctx->tuning.blocks_per_cu;
  if (!per_cu) {
    const int occ = persist_blocks_per_cu(precision, threads);
    per_cu = occ > 0 ? (uint32_t)occ : 1u;
  }
  blocks = (uint32_t)ctx->cus * per_cu;
}

// One persistent launch over passes of one precision (the walker kernel is
// compiled per precision).
static sdd_status run_group(sdd_ctx *ctx, std::vector<Prepared *> &passes, int precision) {
  const uint32_t n = (uint32_t)passes.size();
  if (n == 0) return SDD_OK;
  uint32_t blocks, threads;
  launch_shape(ctx, precision, blocks, threads);
  const uint32_t waves = blocks * (threads / 64);
  BatchScratch B;
  B.d_reqs = ctx->alloc(n * sizeof(DevReq));
  B.d_ctr = ctx->alloc(n * sizeof(uint32_t));
  B.d_done = ctx->alloc(n * sizeof(unsigned long long));
  B.d_ws = ctx->alloc((n + 1) * sizeof(uint32_t));
  if (!B.d_reqs || !B.d_ctr || !B.d_done || !B.d_ws) {
    B.release(ctx);
    return fail(SDD_E_NOMEM, "no workspace left for the batch descriptors");
  }
  std::vector<DevReq> dq(n);
  std::vector<uint32_t> ws(n + 1, 0);
  // waves shared in proportion to paths (work estimate), each request >= 0
  double total = 0.0;
  for (auto *P : passes) total += (double)P->n_paths;
  double acc = 0.0;
  for (uint32_t i = 0; i < n; ++i) {
    dq[i] = passes[i]->dreq;
    dq[i].tile_counter = reinterpret_cast<uint32_t *>(B.d_ctr) + i;
    dq[i].done_counter = reinterpret_cast<unsigned long long *>(B.d_done) + i;
    ws[i] = total > 0 ? (uint32_t)std::llround(acc / total * waves) : 0u;
    acc += (double)passes[i]->n_paths;
  }
  ws[n] = waves;
  sdd_status st = SDD_OK;
  auto check = [&](hipError_t e, const char *what) {
    if (e != hipSuccess && st == SDD_OK) st = fail(SDD_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  };
  check(hipMemcpyAsync(B.d_reqs, dq.data(), n * sizeof(DevReq), hipMemcpyHostToDevice, ctx->stream), "copy reqs");
  check(hipMemcpyAsync(B.d_ws, ws.data(), (n + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, ctx->stream),
        "copy wave shares");
  check(launch_reset(reinterpret_cast<uint32_t *>(B.d_ctr), reinterpret_cast<unsigned long long *>(B.d_done), n,
                     ctx->stream),
        "reset counters");
  if (st == SDD_OK) check(hipEventRecord(ctx->ev[0], ctx->stream), "event");
  if (st == SDD_OK)
    check(launch_walk_persist(precision, reinterpret_cast<const DevReq *>(B.d_reqs), n,
                              reinterpret_cast<const uint32_t *>(B.d_ws), blocks, threads, ctx->stream),
          "walk_persist");
  if (st == SDD_OK) check(hipEventRecord(ctx->ev[1], ctx->stream), "event");
  std::vector<unsigned long long> done(n, 0);
  if (st == SDD_OK)
    check(hipMemcpyAsync(done.data(), B.d_done, n * sizeof(unsigned long long), hipMemcpyDeviceToHost, ctx->stream),
          "copy done");
  if (st == SDD_OK) check(hipStreamSynchronize(ctx->stream), "synchronize");
  B.release(ctx);
  if (st != SDD_OK) return st;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]) == hipSuccess) ctx->stats.last_walk_ms += ms;
  ctx->stats.last_blocks = blocks;
  ctx->stats.last_threads = threads;
  ctx->stats.launches += 1;
  for (auto *P : passes) ctx->stats.last_walk_paths += P->n_paths;
  for (uint32_t i = 0; i < n; ++i)
    if (done[i] != passes[i]->n_paths)
      return fail(SDD_E_DEVICE, "request %u: %llu of %llu paths completed", i, done[i],
                  (unsigned long long)passes[i]->n_paths);
  return SDD_OK;
}

// The walk of a set of passes: one persistent launch per precision present.
static sdd_status run_persistent(sdd_ctx *ctx, std::vector<Prepared *> &passes) {
  ctx->stats.last_walk_ms = 0.0;
  ctx->stats.last_walk_paths = 0;
  for (int prec : {SDD_FP32_MIXED, SDD_FP64}) {
    std::vector<Prepared *> group;
    for (auto *P : passes)
      if ((int)P->dreq.precision == prec) group.push_back(P);
    sdd_status st = run_group(ctx, group, prec);
    if (st != SDD_OK) return st;
  }
  return SDD_OK;
}

static sdd_status run_plain(sdd_ctx *ctx, Prepared &P) {
  char *d_req = ctx->alloc(sizeof(DevReq));
  if (!d_req) return fail(SDD_E_NOMEM, "no workspace left for the request descriptor");
  P.dreq.tile_counter = nullptr;
  P.dreq.done_counter = nullptr;
  sdd_status st = SDD_OK;
  hipError_t e = hipMemcpyAsync(d_req, &P.dreq, sizeof(DevReq), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipEventRecord(ctx->ev[0], ctx->stream);
  for (uint32_t j = 0; j < P.pbeg.size() && e == hipSuccess; ++j)
    e = launch_walk_plain(reinterpret_cast<const DevReq *>(d_req), j, P.pbeg[j], P.pcnt[j], P.rec_off[j],
                          ctx->stream);
  if (e == hipSuccess) e = hipEventRecord(ctx->ev[1], ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) st = fail(SDD_E_DEVICE, "walk_plain: %s", hipGetErrorString(e));
  float ms = 0.f;
  if (st == SDD_OK && hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]) == hipSuccess) {
    ctx->stats.last_walk_ms = ms;
    ctx->stats.last_walk_paths = P.n_paths;
    ctx->stats.launches += P.pbeg.size();
  }
  ctx->release(d_req);
  return st;
}

// Reduce a set of passes' records per node into NodeOut rows (host vector).
// When a pass is the extension of a target-SE request, the node's pilot
// records are the first segment of its reduction.
static sdd_status reduce_passes(sdd_ctx *ctx, std::vector<Prepared *> &passes, std::vector<NodeOut> &out) {
  uint64_t total_nodes = 0;
  for (auto *P : passes) total_nodes += P->pbeg.size();
  out.assign(total_nodes, NodeOut{});
  if (total_nodes == 0) return SDD_OK;
  std::vector<NodeJob> jobs;
  jobs.reserve(total_nodes);
  char *d_out = ctx->alloc(total_nodes * sizeof(NodeOut));
  char *d_jobs = ctx->alloc(total_nodes * sizeof(NodeJob));
  sdd_status st = SDD_OK;
  if (!d_out || !d_jobs) st = fail(SDD_E_NOMEM, "no workspace left for the reduction");
  uint64_t row = 0;
  for (auto *P : passes) {
    for (uint32_t j = 0; j < P->pbeg.size(); ++j, ++row) {
      NodeJob J{};
      J.out = reinterpret_cast<NodeOut *>(d_out) + row;
      const PathRec *ext = reinterpret_cast<const PathRec *>(P->d_recs) + P->rec_off[j];
      if (P->d_recs_pilot) {
        J.recs0 = reinterpret_cast<const PathRec *>(P->d_recs_pilot) + P->pilot_off[j];
        J.count0 = P->pilot_cnt[j];
        J.recs1 = ext;
        J.count1 = P->pcnt[j];
      } else {
        J.recs0 = ext;
        J.count0 = P->pcnt[j];
      }
      jobs.push_back(J);
    }
  }
  if (st == SDD_OK) {
    hipError_t e = hipMemcpyAsync(d_jobs, jobs.data(), jobs.size() * sizeof(NodeJob), hipMemcpyHostToDevice,
                                  ctx->stream);
    if (e == hipSuccess) e = hipEventRecord(ctx->ev[2], ctx->stream);
    if (e == hipSuccess) e = launch_reduce(reinterpret_cast<const NodeJob *>(d_jobs), (uint32_t)jobs.size(),
                                           ctx->stream);
    if (e == hipSuccess) e = hipEventRecord(ctx->ev[3], ctx->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(out.data(), d_out, total_nodes * sizeof(NodeOut), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) st = fail(SDD_E_DEVICE, "reduce: %s", hipGetErrorString(e));
    float ms = 0.f;
    if (st == SDD_OK && hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]) == hipSuccess) ctx->stats.last_reduce_ms = ms;
    if (st == SDD_OK) {
      uint64_t steps = 0;
      for (const NodeOut &o : out) steps += o.steps;
      ctx->stats.last_walk_steps = steps;
    }
  }
  ctx->release(d_out);
  ctx->release(d_jobs);
  return st;
}

// After a pilot pass: decide each node's path count and set up the extension.
static void plan_extension(Prepared &P, const NodeOut *pilot_rows) {
  const uint32_t n = (uint32_t)P.pbeg_all.size();
  double gnorm = 0.0;
  for (size_t k = 0; k + 1 < P.g.size(); k += 2) gnorm = std::max(gnorm, std::hypot(P.g[k], P.g[k + 1]));
  const double target = P.req.target_rel_se * (gnorm > 0 ? gnorm : 1.0);
  P.pilot_off = P.rec_off;
  P.pilot_cnt = P.pcnt;
  for (uint32_t j = 0; j < n; ++j) {
    const NodeOut &o = pilot_rows[j];
    const double s2 = o.var_re + o.var_im;
    double want = std::ceil(s2 / (target * target));
    if (!std::isfinite(want)) want = (double)kMaxTargetPaths;
    uint32_t N = (uint32_t)std::min<double>(std::max<double>(want, (double)kPilotPaths), (double)kMaxTargetPaths);
    P.pcnt_all[j] = N;
    P.pbeg[j] = P.pbeg_all[j] + kPilotPaths;
    P.pcnt[j] = N - kPilotPaths;
  }
  P.pass = 1;
}

static void scatter(const Prepared &P, const NodeOut *rows, sdd_result *res) {
  const uint32_t n = (uint32_t)P.pbeg_all.size();
  for (uint32_t j = 0; j < n; ++j) {
    const NodeOut &o = rows[j];
    if (res->mean) { res->mean[2 * j] = o.mean_re; res->mean[2 * j + 1] = o.mean_im; }
    if (res->var) { res->var[3 * j] = o.var_re; res->var[3 * j + 1] = o.var_im; res->var[3 * j + 2] = o.cov; }
    if (res->se) { res->se[3 * j] = o.se_re; res->se[3 * j + 1] = o.se_im; res->se[3 * j + 2] = o.se; }
    if (res->paths_done) res->paths_done[j] = o.paths_done;
    if (res->steps) res->steps[j] = o.steps;
    if (res->unfinished) res->unfinished[j] = o.unfinished;
    if (res->mean_exit_time) res->mean_exit_time[j] = o.mean_exit_time;
  }
}

static sdd_status copy_records(sdd_ctx *ctx, const Prepared &P, sdd_result *res) {
  if (!res->path_records || P.n_paths == 0) return SDD_OK;
  if (P.req.target_rel_se > 0.0)
    return fail(SDD_E_INVALID, "path_records are available for fixed-path requests only");
  static_assert(sizeof(PathRec) == sizeof(sdd_path_record), "record layout");
  HIP_TRY(hipMemcpyAsync(res->path_records, P.d_recs, P.n_paths * sizeof(PathRec), hipMemcpyDeviceToHost,
                         ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return SDD_OK;
}


// ---------------------------------------------------------------------------
// Execution of prepared requests: one persistent launch for all first passes,
// then (for target-SE requests) one for all extensions.  Caller holds
// ctx->exec.  rows[i] receives request i's per-node results.
// ---------------------------------------------------------------------------
static sdd_status execute(sdd_ctx *ctx, std::vector<Prepared *> &Ps, std::vector<std::vector<NodeOut>> &rows) {
  rows.assign(Ps.size(), {});
  sdd_status st = SDD_OK;
  for (auto *P : Ps) {
    st = upload_pass(ctx, *P);
    if (st != SDD_OK) return st;
  }
  st = run_persistent(ctx, Ps);
  std::vector<NodeOut> all;
  if (st == SDD_OK) st = reduce_passes(ctx, Ps, all);
  if (st != SDD_OK) return st;
  uint64_t row = 0;
  std::vector<Prepared *> ext;
  for (size_t i = 0; i < Ps.size(); ++i) {
    Prepared *P = Ps[i];
    const size_t nn = P->pbeg.size();
    rows[i].assign(all.begin() + row, all.begin() + row + nn);
    row += nn;
    if (P->req.target_rel_se > 0.0) {
      plan_extension(*P, rows[i].data());
      P->d_recs_pilot = P->d_recs;
      P->d_recs = nullptr;
      release_pass(ctx, *P);
      ext.push_back(P);
    }
  }
  if (ext.empty()) return SDD_OK;
  for (auto *P : ext) {
    st = upload_pass(ctx, *P);
    if (st != SDD_OK) return st;
  }
  st = run_persistent(ctx, ext);
  std::vector<NodeOut> erows;
  if (st == SDD_OK) st = reduce_passes(ctx, ext, erows);
  if (st != SDD_OK) return st;
  row = 0;
  for (size_t i = 0, e = 0; i < Ps.size() && e < ext.size(); ++i) {
    if (Ps[i] != ext[e]) continue;
    const size_t nn = Ps[i]->pbeg.size();
    rows[i].assign(erows.begin() + row, erows.begin() + row + nn);
    row += nn;
    ++e;
  }
  return SDD_OK;
}

// Workspace a request needs while it runs (upper bound for target-SE
// requests, whose extension size is known only after the pilot).
static uint64_t footprint(sdd_ctx *ctx, Prepared &P) {
  build_tiles(P, ctx->tuning.tile_paths ? ctx->tuning.tile_paths : 512u);
  const uint64_t n = P.pbeg.size();
  uint64_t b = pass_bytes(P) + Arena::round(n * (sizeof(NodeOut) + sizeof(NodeJob))) + 4 * 1024 +
               Arena::round(sizeof(DevReq) * 2);
  if (P.req.target_rel_se > 0.0) b += Arena::round(n * (uint64_t)kMaxTargetPaths * sizeof(PathRec));
  return b;
}

// ---------------------------------------------------------------------------
// Served mode: a worker thread admits queued requests while the workspace
// has room and runs the admitted set together.
// ---------------------------------------------------------------------------
static void finish_ticket(sdd_ctx *ctx, Ticket &T, sdd_status st, const char *err) {
  // caller holds ctx->mu
  T.status = T.cancelled ? SDD_E_CANCELLED : st;
  if (err) T.error = err;
  T.done = true;
}

static void worker_main(sdd_ctx *ctx) {
  hipSetDevice(ctx->device);
  for (;;) {
    std::vector<std::shared_ptr<Ticket>> batch;
    {
      std::unique_lock<std::mutex> lk(ctx->mu);
      ctx->cv.wait(lk, [&] { return ctx->stop || !ctx->queue.empty(); });
      if (ctx->stop) {
        for (auto &T : ctx->queue) {
          T->cancelled = true;
          finish_ticket(ctx, *T, SDD_E_CANCELLED, "context destroyed");
          T->P.reset();
        }
        ctx->queue.clear();
        ctx->done_cv.notify_all();
        return;
      }
      // admission by workspace: FIFO while the footprints fit
      uint64_t room = ctx->arena.largest_free();
      while (!ctx->queue.empty()) {
        auto T = ctx->queue.front();
        lk.unlock();
        const uint64_t need = footprint(ctx, *T->P);
        lk.lock();
        if (need > ctx->arena.size()) {
          ctx->queue.pop_front();
          finish_ticket(ctx, *T, SDD_E_NOMEM, "request can never fit in the workspace");
          T->P.reset();
          continue;
        }
        if (need > room && !batch.empty()) break;
        if (need > room) break;   // wait for memory held by blocking callers
        room -= need;
        batch.push_back(T);
        ctx->queue.pop_front();
      }
    }
    if (batch.empty()) {
      std::this_thread::sleep_for(std::chrono::milliseconds(1));
      continue;
    }
    std::vector<Prepared *> Ps;
    for (auto &T : batch) Ps.push_back(T->P.get());
    std::vector<std::vector<NodeOut>> rows;
    sdd_status st;
    std::string err;
    {
      std::lock_guard<std::mutex> ex(ctx->exec);
      st = execute(ctx, Ps, rows);
      if (st != SDD_OK) err = g_last_error;
      for (size_t i = 0; i < batch.size() && st == SDD_OK; ++i) {
        if (batch[i]->cancelled) continue;
        scatter(*Ps[i], rows[i].data(), &batch[i]->res);
        sdd_status s2 = copy_records(ctx, *Ps[i], &batch[i]->res);
        if (s2 != SDD_OK) { st = s2; err = g_last_error; }
      }
      for (auto *P : Ps) release_all(ctx, *P);
    }
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      for (auto &T : batch) {
        finish_ticket(ctx, *T, st, st == SDD_OK ? nullptr : err.c_str());
        T->P.reset();
      }
    }
    ctx->done_cv.notify_all();
  }
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *sdd_status_string(sdd_status s) {
  switch (s) {
    case SDD_OK: return "ok";
    case SDD_E_INVALID: return "invalid argument";
    case SDD_E_NOMEM: return "workspace exhausted";
    case SDD_E_DEVICE: return "device error";
    case SDD_E_BUSY: return "busy";
    case SDD_E_NOTFOUND: return "not found";
    case SDD_E_TIMEOUT: return "timeout";
    case SDD_E_CANCELLED: return "cancelled";
  }
  return "unknown status";
}

const char *sdd_last_error(void) { return g_last_error.c_str(); }

sdd_status sdd_create(int device, void *workspace_dev, size_t workspace_bytes, void *hip_stream,
                      sdd_ctx_t *out) {
  if (!out) return fail(SDD_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!workspace_dev || workspace_bytes < 4096)
    return fail(SDD_E_INVALID, "a device workspace of at least 4096 bytes is required");
  if (((uintptr_t)workspace_dev & 255u) != 0) return fail(SDD_E_INVALID, "workspace must be 256-byte aligned");
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(SDD_E_INVALID, "device %d out of range (%d devices)", device, ndev);
  HIP_TRY(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(SDD_E_DEVICE, "device %d is %s; this library is built for gfx950", device, prop.gcnArchName);
  auto ctx = std::make_unique<sdd_ctx>();
  for (auto &e : ctx->ev) HIP_TRY(hipEventCreate(&e));
  ctx->device = device;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  ctx->cus = prop.multiProcessorCount;
  ctx->arena.init(reinterpret_cast<char *>(workspace_dev), workspace_bytes);
  *out = ctx.release();
  return SDD_OK;
}

sdd_status sdd_destroy(sdd_ctx_t ctx) {
  if (!ctx) return fail(SDD_E_INVALID, "ctx is NULL");
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->stop = true;
  }
  ctx->cv.notify_all();
  if (ctx->worker.joinable()) ctx->worker.join();
  {
    std::lock_guard<std::mutex> ex(ctx->exec);   // no blocking call still running
    for (auto &e : ctx->ev)
      if (e) hipEventDestroy(e);
  }
  delete ctx;
  return SDD_OK;
}

sdd_status sdd_model_create(sdd_ctx_t ctx, const sdd_model_desc *d, sdd_model_t *out) {
  if (!ctx || !d || !out) return fail(SDD_E_INVALID, "NULL argument");
  if (!(d->y_lo < d->y_hi) || !(d->z_lo < d->z_hi) || !std::isfinite(d->y_lo) || !std::isfinite(d->y_hi) ||
      !std::isfinite(d->z_lo) || !std::isfinite(d->z_hi))
    return fail(SDD_E_INVALID, "domain must satisfy y_lo < y_hi and z_lo < z_hi (finite)");
  if (d->n_regions > SDD_MAX_REGIONS) return fail(SDD_E_INVALID, "at most %d regions", SDD_MAX_REGIONS);
  if (d->n_regions && !d->regions) return fail(SDD_E_INVALID, "regions is NULL");
  if (!(d->sigma_background >= 0.0) || !std::isfinite(d->sigma_background))
    return fail(SDD_E_INVALID, "sigma_background must be finite and >= 0");
  if (!(d->length_unit_m > 0.0) || !std::isfinite(d->length_unit_m))
    return fail(SDD_E_INVALID, "length_unit_m must be > 0");
  for (uint32_t k = 0; k < d->n_regions; ++k) {
    const sdd_region &r = d->regions[k];
    if (r.kind < SDD_HALF_Z_LT || r.kind > SDD_TRIANGLE) return fail(SDD_E_INVALID, "region %u: bad kind", k);
    if (!(r.sigma >= 0.0) || !std::isfinite(r.sigma)) return fail(SDD_E_INVALID, "region %u: bad sigma", k);
    for (double v : r.v)
      if (!std::isfinite(v)) return fail(SDD_E_INVALID, "region %u: non-finite geometry", k);
  }
  auto m = std::make_unique<HostModel>();
  m->desc = *d;
  m->regions.assign(d->regions, d->regions + d->n_regions);
  m->desc.regions = nullptr;
  DevModel dm;
  std::memset(&dm, 0, sizeof(dm));
  dm.nprims = (int32_t)d->n_regions;
  for (uint32_t k = 0; k < d->n_regions; ++k) {
    dm.kind[k] = d->regions[k].kind;
    for (int i = 0; i < 6; ++i) {
      dm.pd[k][i] = d->regions[k].v[i];
      dm.pf[k][i] = (float)d->regions[k].v[i];
    }
    dm.sigma[k] = d->regions[k].sigma;
  }
  dm.sigma[d->n_regions] = d->sigma_background;
  dm.y_lo = d->y_lo; dm.y_hi = d->y_hi; dm.z_lo = d->z_lo; dm.z_hi = d->z_hi;
  dm.length_unit_m = d->length_unit_m;
  m->dev = ctx->alloc(sizeof(DevModel));
  if (!m->dev) return fail(SDD_E_NOMEM, "no workspace left for the model");
  {
    std::lock_guard<std::mutex> ex(ctx->exec);
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipMemcpyAsync(m->dev, &dm, sizeof(dm), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      ctx->release(m->dev);
      return fail(SDD_E_DEVICE, "model upload: %s", hipGetErrorString(e));
    }
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  const uint32_t id = ctx->next_model++;
  ctx->models[id] = std::move(m);
  *out = id;
  return SDD_OK;
}

sdd_status sdd_model_destroy(sdd_ctx_t ctx, sdd_model_t model) {
  if (!ctx) return fail(SDD_E_INVALID, "ctx is NULL");
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->models.find(model);
  if (it == ctx->models.end()) return fail(SDD_E_NOTFOUND, "unknown model %u", model);
  const int busy = it->second->in_flight.load();
  if (busy > 0) return fail(SDD_E_BUSY, "model %u is used by %d requests in flight", model, busy);
  ctx->arena.release(it->second->dev);
  ctx->models.erase(it);
  return SDD_OK;
}

sdd_status sdd_solve(sdd_ctx_t ctx, const sdd_request *req, sdd_result *res) {
  return sdd_solve_batch(ctx, 1, req, res);
}

sdd_status sdd_solve_batch(sdd_ctx_t ctx, uint32_t n, const sdd_request *reqs, sdd_result *res) {
  if (!ctx) return fail(SDD_E_INVALID, "ctx is NULL");
  if (n && (!reqs || !res)) return fail(SDD_E_INVALID, "NULL requests or results");
  std::vector<std::unique_ptr<Prepared>> own(n);
  for (uint32_t i = 0; i < n; ++i) {
    if (!res[i].mean && reqs[i].n_nodes) return fail(SDD_E_INVALID, "result %u: mean is NULL", i);
    if (res[i].path_records && reqs[i].target_rel_se > 0.0)
      return fail(SDD_E_INVALID, "result %u: path_records need a fixed-path request", i);
    sdd_status st = prepare(ctx, &reqs[i], own[i]);
    if (st != SDD_OK) return st;
  }
  std::lock_guard<std::mutex> ex(ctx->exec);
  HIP_TRY(hipSetDevice(ctx->device));
  std::vector<Prepared *> Ps;
  for (auto &P : own) Ps.push_back(P.get());
  std::vector<std::vector<NodeOut>> rows;
  sdd_status st = execute(ctx, Ps, rows);
  for (uint32_t i = 0; i < n && st == SDD_OK; ++i) {
    scatter(*Ps[i], rows[i].data(), &res[i]);
    st = copy_records(ctx, *Ps[i], &res[i]);
  }
  for (auto *P : Ps) release_all(ctx, *P);
  return st;
}

sdd_status sdd_solve_plain(sdd_ctx_t ctx, const sdd_request *req, sdd_result *res) {
  if (!ctx || !req || !res) return fail(SDD_E_INVALID, "NULL argument");
  if (req->target_rel_se > 0.0) return fail(SDD_E_INVALID, "the plain form takes fixed path counts");
  if (!res->mean && req->n_nodes) return fail(SDD_E_INVALID, "result mean is NULL");
  std::unique_ptr<Prepared> P;
  sdd_status st = prepare(ctx, req, P);
  if (st != SDD_OK) return st;
  P->dreq.precision = SDD_FP64;
  std::lock_guard<std::mutex> ex(ctx->exec);
  HIP_TRY(hipSetDevice(ctx->device));
  st = upload_pass(ctx, *P);
  if (st != SDD_OK) return st;
  st = run_plain(ctx, *P);
  std::vector<Prepared *> passes{P.get()};
  std::vector<NodeOut> rows;
  if (st == SDD_OK) st = reduce_passes(ctx, passes, rows);
  if (st == SDD_OK) {
    scatter(*P, rows.data(), res);
    st = copy_records(ctx, *P, res);
  }
  release_all(ctx, *P);
  return st;
}

sdd_status sdd_submit(sdd_ctx_t ctx, const sdd_request *req, sdd_result *res, sdd_ticket_t *out) {
  if (!ctx || !req || !res || !out) return fail(SDD_E_INVALID, "NULL argument");
  if (!res->mean && req->n_nodes) return fail(SDD_E_INVALID, "result mean is NULL");
  if (res->path_records && req->target_rel_se > 0.0)
    return fail(SDD_E_INVALID, "path_records need a fixed-path request");
  auto T = std::make_shared<Ticket>();
  sdd_status st = prepare(ctx, req, T->P);
  if (st != SDD_OK) return st;
  T->res = *res;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->stop) return fail(SDD_E_INVALID, "context is shutting down");
    const uint64_t id = ctx->next_ticket++;
    ctx->tickets[id] = T;
    ctx->queue.push_back(T);
    if (!ctx->worker.joinable()) ctx->worker = std::thread(worker_main, ctx);
    *out = id;
  }
  ctx->cv.notify_all();
  return SDD_OK;
}

static sdd_status take_result(sdd_ctx *ctx, uint64_t id, Ticket &T) {
  // caller holds ctx->mu; the ticket is finished
  const sdd_status st = T.status;
  if (st != SDD_OK && st != SDD_E_CANCELLED) fail(st, "%s", T.error.c_str());
  if (st == SDD_E_CANCELLED) fail(st, "ticket %llu was cancelled", (unsigned long long)id);
  ctx->tickets.erase(id);
  return st;
}

sdd_status sdd_poll(sdd_ctx_t ctx, sdd_ticket_t t, int *done) {
  if (!ctx || !done) return fail(SDD_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->tickets.find(t);
  if (it == ctx->tickets.end()) return fail(SDD_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)t);
  *done = it->second->done ? 1 : 0;
  if (!it->second->done) return SDD_OK;
  auto T = it->second;
  return take_result(ctx, t, *T);
}

sdd_status sdd_wait(sdd_ctx_t ctx, sdd_ticket_t t, int64_t timeout_ns) {
  if (!ctx) return fail(SDD_E_INVALID, "ctx is NULL");
  std::unique_lock<std::mutex> lk(ctx->mu);
  auto it = ctx->tickets.find(t);
  if (it == ctx->tickets.end()) return fail(SDD_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)t);
  auto T = it->second;
  if (timeout_ns < 0) {
    ctx->done_cv.wait(lk, [&] { return T->done; });
  } else if (!ctx->done_cv.wait_for(lk, std::chrono::nanoseconds(timeout_ns), [&] { return T->done; })) {
    return fail(SDD_E_TIMEOUT, "ticket %llu not finished", (unsigned long long)t);
  }
  return take_result(ctx, t, *T);
}

sdd_status sdd_cancel(sdd_ctx_t ctx, sdd_ticket_t t) {
  if (!ctx) return fail(SDD_E_INVALID, "ctx is NULL");
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->tickets.find(t);
  if (it == ctx->tickets.end()) return fail(SDD_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)t);
  auto T = it->second;
  if (T->done) return fail(SDD_E_BUSY, "ticket %llu already finished", (unsigned long long)t);
  T->cancelled = true;
  auto q = std::find(ctx->queue.begin(), ctx->queue.end(), T);
  if (q != ctx->queue.end()) {   // not admitted yet: finish it now
    ctx->queue.erase(q);
    finish_ticket(ctx, *T, SDD_E_CANCELLED, nullptr);
    T->P.reset();
    ctx->done_cv.notify_all();
  }
  return SDD_OK;
}

sdd_status sdd_request_footprint(sdd_ctx_t ctx, const sdd_request *req, uint64_t *bytes) {
  if (!ctx || !req || !bytes) return fail(SDD_E_INVALID, "NULL argument");
  std::unique_ptr<Prepared> P;
  sdd_status st = prepare(ctx, req, P);
  if (st != SDD_OK) return st;
  *bytes = footprint(ctx, *P);
  return SDD_OK;
}

sdd_status sdd_set_tuning(sdd_ctx_t ctx, const sdd_tuning *t) {
  if (!ctx || !t) return fail(SDD_E_INVALID, "NULL argument");
  if (t->block_threads && (t->block_threads % 64 || t->block_threads > 256))
    return fail(SDD_E_INVALID, "block_threads must be a multiple of 64, at most 256 (the walker's launch bound)");
  if (t->blocks_per_cu > 64) return fail(SDD_E_INVALID, "blocks_per_cu at most 64");
  if (t->tile_paths > (1u << 24)) return fail(SDD_E_INVALID, "tile_paths at most 2^24");
  std::lock_guard<std::mutex> ex(ctx->exec);
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->tuning = *t;
  if (!ctx->tuning.block_threads) ctx->tuning.block_threads = 256;
  if (!ctx->tuning.tile_paths) ctx->tuning.tile_paths = 512;
  if (!ctx->tuning.slice_iters) ctx->tuning.slice_iters = 4096;
  return SDD_OK;
}

sdd_status sdd_get_stats(sdd_ctx_t ctx, sdd_stats *out) {
  if (!ctx || !out) return fail(SDD_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> ex(ctx->exec);
  *out = ctx->stats;
  return SDD_OK;
}

sdd_status sdd_get_tuning(sdd_ctx_t ctx, sdd_tuning *t) {
  if (!ctx || !t) return fail(SDD_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(ctx->mu);
  *t = ctx->tuning;
  return SDD_OK;
}

}  // extern "C"
