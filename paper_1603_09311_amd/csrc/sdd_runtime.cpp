// Host runtime behind the C ABI declared in include/sdd.h: context,
// workspace allocator (the caller's device buffer is the only device memory
// used), resident models, request preparation, batched persistent launches,
// the plain per-node form and the served (continuous-batching) loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
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
hipError_t launch_walk_persist(int precision, int sig, const DevReq *reqs_dev, uint32_t n_req,
                               const uint32_t *wave_start_dev, uint32_t budget, uint32_t refill_mask, uint32_t blocks,
                               uint32_t threads, uint32_t lds_bytes, hipStream_t st);
hipError_t launch_reduce(const NodeJob *jobs_dev, uint32_t n_jobs, hipStream_t st);
hipError_t launch_reduce_fanout(const FanJob *jobs_dev, uint32_t n_jobs, int M, double y_lo, double y_hi, double z_lo,
                                double z_hi, hipStream_t st);
hipError_t launch_reset(uint32_t *tile_counters, unsigned long long *done, uint32_t n, hipStream_t st);
int persist_blocks_per_cu(int precision, int sig, uint32_t threads, uint32_t lds_bytes);
uint32_t lds_walker_threads();
hipError_t launch_walk_kappa(int precision, const KReq *req_dev, uint32_t blocks, hipStream_t st);
int kappa_blocks_per_cu(int precision);
uint32_t kappa_threads();
hipError_t scratch_init(int device, void **out);
size_t scratch_bytes();
std::mutex &scratch_lock(int device);
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

// for the host sub-domain solver (its own translation unit)
sdd_status sdd_rbffd_fail(sdd_status st, const char *msg) { return fail(st, "%s", msg); }

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
  std::vector<SigmaCell> grid;     // sigma grid (FP32 generic signature), empty if none
  std::vector<SigmaCell> grid_ext; // its two-line cells' extension entries
  std::vector<uint8_t> lds;        // its LDS form (class table, class bytes), empty if none
  // device allocations
  char *d_g = nullptr, *d_nodes = nullptr, *d_tiles = nullptr, *d_recs = nullptr;
  char *d_grid = nullptr, *d_grid_ext = nullptr, *d_lds = nullptr;
  char *d_recs_pilot = nullptr;    // pilot records kept for the final reduction
  std::vector<uint64_t> pilot_off; // per node pilot record offset
  std::vector<uint32_t> pilot_cnt;
  int pass = 0;                    // 0 fixed/pilot, 1 extension
  uint32_t slot = 0;               // done-counter slot in a prepared batch
};

struct Ticket {
  std::unique_ptr<Prepared> P;
  sdd_result res{};
  sdd_status status = SDD_OK;
  bool done = false, cancelled = false;
  bool waited = false;             // admission once had to wait for workspace
  std::string error;
};

struct sdd_ctx;

// exec for a caller thread.  The served worker takes exec once per slice and
// gives way to any caller waiting for it (std::mutex promises no fairness).
struct ExecGuard {
  explicit ExecGuard(sdd_ctx *ctx);
  ~ExecGuard();
  sdd_ctx *ctx;
};

struct sdd_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  Arena arena;
  int cus = 0;
  size_t lds_per_block = 0;        // the device's LDS limit per block (the LDS-grid walker)
  sdd_tuning tuning{256, 0, 512, 4096, 1};
  std::mutex exec;                 // one launch sequence at a time on the stream
  std::atomic<int> exec_waiters{0};   // callers (not the served worker) waiting for exec
  std::mutex mu;                   // guards everything below and the arena
  char *alloc(size_t b) {
    std::lock_guard<std::mutex> lk(mu);
    return arena.alloc(b);
  }
  // Every release moves the memory epoch and wakes the served worker, which
  // may be waiting for workspace to admit a request.
  void release(char *p) {
    if (!p) return;
    {
      std::lock_guard<std::mutex> lk(mu);
      arena.release(p);
      ++epoch;
    }
    cv.notify_all();
  }
  uint64_t epoch = 0;              // bumped by every release, submit, cancel and stop
  uint64_t held_long = 0;          // workspace held by resident models and prepared batches
  uint64_t reserved = 0;           // workspace promised to served flights
  uint32_t served_in_flight_max = 0, served_waits = 0, served_requeues = 0;
  double served_walk_ms = 0.0;     // summed slice times (worker thread only)
  uint64_t served_slices = 0;
  std::unordered_map<uint32_t, std::unique_ptr<HostModel>> models;
  uint32_t next_model = 1;
  // served mode
  std::unordered_map<uint64_t, std::shared_ptr<Ticket>> tickets;
  std::deque<std::shared_ptr<Ticket>> queue;
  // target-SE flights whose extension did not fit next to the others: they
  // gave their workspace back and walk all their paths in one pass once
  // admitted again (ahead of the queue)
  std::deque<std::shared_ptr<Ticket>> requeue;
  uint64_t next_ticket = 1;
  std::condition_variable cv, done_cv;
  std::thread worker;
  bool stop = false;
  // timing of the last walk / reduction launches (guarded by exec)
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  sdd_stats stats{};
  char *scratch = nullptr;         // this device's static scratch (sdd_solve_noalloc)
  bool debug = false;              // SDD_DEBUG=1: per-slice trace of the served loop on stderr
};

ExecGuard::ExecGuard(sdd_ctx *c) : ctx(c) {
  ctx->exec_waiters.fetch_add(1);
  ctx->exec.lock();
  ctx->exec_waiters.fetch_sub(1);
}
ExecGuard::~ExecGuard() { ctx->exec.unlock(); }

// exec for the served worker: first let every waiting caller through.
static std::unique_lock<std::mutex> worker_exec(sdd_ctx *ctx) {
  while (ctx->exec_waiters.load() > 0) std::this_thread::yield();
  return std::unique_lock<std::mutex>(ctx->exec);
}

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
  if (r->flags & ~(uint32_t)(SDD_FLAG_NO_SIGMA_GRID | SDD_FLAG_EXIT_NAIVE | SDD_FLAG_NO_LDS_GRID))
    return fail(SDD_E_INVALID, "unknown flags");
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

// ---------------------------------------------------------------------------
// Sigma grid of the FP32 walk's generic signature (SigmaCell).  Each cell is
// classified against every inequality of every primitive over the cell grown
// by a margin (1e-3 of its width; the FP32 cell index errs by at most about
// 1.5e-5 of a width), and each inequality's edge function only where its sign
// holds with a margin (4 2^-24 times the magnitude of its terms) above the
// rounding of its FP32 evaluation.  So for every FP32 point the kernel maps to
// a cell, the cell's answer is the primitive loop's.
// ---------------------------------------------------------------------------
namespace {
struct GLine {
  float A, B, C;   // e = fma(A, a, fma(B, b, C)) in FP32
  uint32_t mode;   // 0: in iff e < 0, 1: in iff e >= 0
};
enum GSign { kGNeg, kGPos, kGCross };
enum GStat { kGOut, kGIn, kGOne };

// The primitive's inequalities as lines, in the primitive loop's FP32
// expressions (parameters relative to the centre): a half-plane or box side
// a < y0 is e = fl(a - y0) < 0 (A = 1, B = 0, C = -y0: the inner fma gives
// -y0 exactly), whose sign is the compare's; a triangle edge is its oriented
// (A, B, C).
int prim_lines(int kind, const float *v, GLine *L) {
  switch (kind) {
    case SDD_HALF_Z_LT: L[0] = {0.f, 1.f, -v[0], 0u}; return 1;   // b < z0
    case SDD_HALF_Y_LT: L[0] = {1.f, 0.f, -v[0], 0u}; return 1;   // a < y0
    case SDD_BOX:
      L[0] = {1.f, 0.f, -v[0], 1u};   // a >= y0
      L[1] = {1.f, 0.f, -v[1], 0u};   // a < y1
      L[2] = {0.f, 1.f, -v[2], 1u};   // b >= z0
      L[3] = {0.f, 1.f, -v[3], 0u};   // b < z1
      return 4;
    default:   // triangle edge m, oriented: the interior is e >= 0 on all three
      for (int m = 0; m < 3; ++m) L[m] = {v[3 * m], v[3 * m + 1], v[3 * m + 2], 1u};
      return 3;
  }
}

// Sign of the line over a cell (its corners: e is linear).  The FP32 value
// fma(A, a, fma(B, b, C)) is within 2u (|A a| + |B b| + |C|)(1 + u) of
// A a + B b + C (two roundings, u = 2^-24), so a sign is certain beyond
// 4u times that magnitude.
GSign classify(const GLine &L, double a0, double a1, double b0, double b1) {
  double emin = HUGE_VAL, emax = -HUGE_VAL, mag = 0.0;
  const double as[2] = {a0, a1}, bs[2] = {b0, b1};
  const double A = L.A, B = L.B, C = L.C;
  for (double a : as)
    for (double b : bs) {
      const double e = A * a + B * b + C;
      emin = std::min(emin, e);
      emax = std::max(emax, e);
      mag = std::max(mag, std::fabs(A * a) + std::fabs(B * b) + std::fabs(C));
    }
  const double m = 4.0 * 0x1p-24 * mag;
  if (emin > m) return kGPos;
  if (emax < -m) return kGNeg;
  return kGCross;
}

// One test of a point against a line: t = (e >= 0), e the edge function, and
// the primitive's condition is t (inv = false) or not t (inv = true).  The
// loop's two tests read: e >= 0 (t: a box's lower sides, a triangle's oriented
// edges), e < 0 (not t: half-planes, a box's upper sides).
struct LineTest {
  GLine line;
  bool inv;
};

// A primitive over a cell: outside everywhere, inside everywhere, or inside
// iff every one of its crossing tests holds (n of them).
struct PrimCell {
  int status;   // kGOut, kGIn, or kGOne for a conjunction of tests
  int n;
  LineTest t[4];
};

PrimCell prim_cell(const GLine *L, int nl, double a0, double a1, double b0, double b1) {
  PrimCell P{kGOut, 0, {}};
  GSign c[4];
  for (int i = 0; i < nl; ++i) c[i] = classify(L[i], a0, a1, b0, b1);
  for (int i = 0; i < nl; ++i) {
    const bool holds = L[i].mode == 0u ? c[i] == kGNeg : c[i] == kGPos;
    const bool fails = L[i].mode == 0u ? c[i] == kGPos : c[i] == kGNeg;
    if (fails) return P;
    if (!holds) P.t[P.n++] = LineTest{L[i], L[i].mode == 0u};
  }
  P.status = P.n == 0 ? kGIn : kGOne;
  return P;
}

bool same_line(const LineTest &x, const LineTest &y) {
  return x.line.A == y.line.A && x.line.B == y.line.B && x.line.C == y.line.C;
}
}  // namespace

static constexpr uint32_t kGridCells = 65536;

// The cell's line in SigmaCell form.
static void put_line(SigmaCell &C, const LineTest &t) {
  C.A = t.line.A;
  C.B = t.line.B;
  C.C = t.line.C;
}

// Sigma grid of the FP32 walk's generic signature.  Per cell: the primitives
// in list order up to the first one that holds on the whole cell; those that
// cross it are conjunctions of line tests; if all their tests use at most two
// distinct lines, the cell's increment is a function of the two signs
// (e1 >= 0, e2 >= 0), evaluated for the four combinations with the
// primitives' first-match rule.  Cells with more lines take the primitive
// loop.  Two-line cells keep their second line and the increments of
// e2 >= 0 in an entry of `ext`.
static void build_sigma_grid(DevReq &q, std::vector<SigmaCell> &grid, std::vector<SigmaCell> &ext) {
  const int np = (int)q.nprims;
  GLine lines[kMaxPrims][4];
  int nl[kMaxPrims];
  for (int k = 0; k < np; ++k) nl[k] = prim_lines(q.kind[k], q.pf[k], lines[k]);
  // cells about square, at most kGridCells
  const double hy = q.fhy, hz = q.fhz;
  uint32_t gy, gz;
  if (hy >= hz) {
    gy = 256;
    gz = (uint32_t)std::max(1.0, std::min(256.0, std::floor(256.0 * hz / hy)));
  } else {
    gz = 256;
    gy = (uint32_t)std::max(1.0, std::min(256.0, std::floor(256.0 * hy / hz)));
  }
  q.gy = gy;
  q.gz = gz;
  q.gmy = (float)(gy - 1);
  q.gmz = (float)(gz - 1);
  q.gsy = (float)((double)gy / (2.0 * hy));
  q.goy = (float)(hy * (double)q.gsy);
  q.gsz = (float)((double)gz / (2.0 * hz));
  q.goz = (float)(hz * (double)q.gsz);
  grid.assign((size_t)gy * gz, SigmaCell{});
  ext.clear();
  std::map<std::vector<uint8_t>, uint32_t> ext_index;
  PrimCell pc[kMaxPrims];
  for (uint32_t j = 0; j < gz; ++j) {
    // the points the kernel maps to row j: j <= b gsz + goz < j + 1
    const double b0 = ((double)j - (double)q.goz) / (double)q.gsz;
    const double b1 = ((double)j + 1.0 - (double)q.goz) / (double)q.gsz;
    const double db = 1e-3 * (b1 - b0);
    for (uint32_t i = 0; i < gy; ++i) {
      const double a0 = ((double)i - (double)q.goy) / (double)q.gsy;
      const double a1 = ((double)i + 1.0 - (double)q.goy) / (double)q.gsy;
      const double da = 1e-3 * (a1 - a0);
      SigmaCell &C = grid[(size_t)j * gy + i];
      // the primitives that matter, and the distinct lines their tests use
      int last = np;   // first primitive holding on the whole cell (np: none)
      bool loop = false;
      LineTest L[2];
      int nlines = 0;
      for (int k = 0; k < np && !loop; ++k) {
        pc[k] = prim_cell(lines[k], nl[k], a0 - da, a1 + da, b0 - db, b1 + db);
        if (pc[k].status == kGIn) { last = k; break; }
        for (int m = 0; m < pc[k].n && !loop; ++m) {
          int f = -1;
          for (int l = 0; l < nlines; ++l)
            if (same_line(L[l], pc[k].t[m])) f = l;
          if (f < 0) {
            if (nlines == 2) loop = true;
            else L[nlines++] = pc[k].t[m];
          }
        }
      }
      if (loop) {
        C.inc_ge = kCellLoop;
        continue;
      }
      // the increment for each sign combination (t1, t2): the first primitive
      // (up to `last`) whose tests all hold, else `last`'s region (the
      // background when last == np)
      uint32_t T[4];
      for (int combo = 0; combo < 4; ++combo) {
        const bool t[2] = {(combo & 1) != 0, (combo & 2) != 0};
        int region = last;
        for (int k = 0; k < last; ++k) {
          if (pc[k].status != kGOne) continue;
          bool all = true;
          for (int m = 0; m < pc[k].n; ++m) {
            const LineTest &x = pc[k].t[m];
            const int l = same_line(L[0], x) ? 0 : 1;
            all = all && (t[l] != x.inv);
          }
          if (all) { region = k; break; }
        }
        T[combo] = q.cfx[region];
      }
      if (nlines == 0) {
        C.A = C.B = C.C = 0.f;   // e = +0 >= 0
        C.inc_ge = C.inc_lt = T[0];
      } else if (nlines == 1 || (T[0] == T[2] && T[1] == T[3])) {
        put_line(C, L[0]);
        C.inc_ge = T[1];
        C.inc_lt = T[0];
      } else {
        put_line(C, L[0]);
        C.inc_ge = T[1] | kCellTwo;
        C.inc_lt = T[0];
        SigmaCell E{};
        put_line(E, L[1]);
        E.inc_ge = T[3];   // e1 >= 0, e2 >= 0
        E.inc_lt = T[2];   // e1 < 0, e2 >= 0
        const uint8_t *eb = reinterpret_cast<const uint8_t *>(&E);
        std::vector<uint8_t> key(eb, eb + sizeof(E));
        auto it = ext_index.find(key);
        if (it == ext_index.end()) {
          it = ext_index.emplace(key, (uint32_t)ext.size()).first;
          ext.push_back(E);
        }
        C.xi = it->second;
      }
    }
  }
}

// The LDS form of a sigma grid: one class byte per cell (padded to 16 bytes),
// then from byte `table` the grid's distinct cells once (a class table) and
// the two-line cells' extension entries (each cell's xi renumbered to its
// entry's place in this table); empty when the grid has more than
// kMaxLdsClasses distinct cells or the form would not fit in max_bytes of
// LDS.  Padded to a multiple of 16 bytes.
static void build_lds_form(const std::vector<SigmaCell> &grid, const std::vector<SigmaCell> &ext, size_t max_bytes,
                           std::vector<uint8_t> &out, uint32_t &table) {
  out.clear();
  table = 0;
  std::vector<SigmaCell> classes;
  std::map<std::vector<uint8_t>, uint32_t> index;
  std::vector<uint8_t> ids(grid.size());
  for (size_t c = 0; c < grid.size(); ++c) {
    const uint8_t *b = reinterpret_cast<const uint8_t *>(&grid[c]);
    std::vector<uint8_t> key(b, b + sizeof(SigmaCell));
    auto it = index.find(key);
    if (it == index.end()) {
      if (classes.size() == kMaxLdsClasses) return;
      it = index.emplace(key, (uint32_t)classes.size()).first;
      classes.push_back(grid[c]);
    }
    ids[c] = (uint8_t)it->second;
  }
  for (SigmaCell &C : classes)
    if ((C.inc_ge & kCellFlags) == kCellTwo) C.xi += (uint32_t)classes.size();
  const size_t off = (ids.size() + 15) / 16 * 16;
  const size_t n = classes.size() + ext.size();
  const size_t bytes = off + n * sizeof(SigmaCell);
  if (bytes > max_bytes) return;
  table = (uint32_t)off;
  out.assign(bytes, 0);
  std::memcpy(out.data(), ids.data(), ids.size());
  std::memcpy(out.data() + off, classes.data(), classes.size() * sizeof(SigmaCell));
  if (!ext.empty()) std::memcpy(out.data() + off + classes.size() * sizeof(SigmaCell), ext.data(), ext.size() * sizeof(SigmaCell));
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
  // the FP32 walk measures positions from the centre of the domain, in units
  // of K = sqrt(dt) sqrt(2 ln 2) (the step length per sqrt(-log2 u))
  q.ymid = 0.5 * (q.y_lo + q.y_hi);
  q.zmid = 0.5 * (q.z_lo + q.z_hi);
  q.kscale = q.s * std::sqrt(2.0 * std::log(2.0));
  q.kinv = 1.0 / q.kscale;
  const double ki = q.kinv;
  const uint32_t np = (uint32_t)m.regions.size();
  q.nprims = np;
  for (uint32_t k = 0; k < np; ++k) {
    q.c[k] = alpha_of(r, m, m.regions[k].sigma) * r.dt / 2.0;
    q.kind[k] = m.regions[k].kind;
    const double *v = m.regions[k].v;
    for (int i = 0; i < 6; ++i) q.pd[k][i] = v[i];
    // centred FP32 geometry in units of K: (y - ymid) / K, (z - zmid) / K
    switch (m.regions[k].kind) {
      case SDD_HALF_Z_LT: q.pf[k][0] = (float)((v[0] - q.zmid) * ki); break;
      case SDD_HALF_Y_LT: q.pf[k][0] = (float)((v[0] - q.ymid) * ki); break;
      case SDD_BOX:
        q.pf[k][0] = (float)((v[0] - q.ymid) * ki); q.pf[k][1] = (float)((v[1] - q.ymid) * ki);
        q.pf[k][2] = (float)((v[2] - q.zmid) * ki); q.pf[k][3] = (float)((v[3] - q.zmid) * ki);
        break;
      default: {
        // edge e from vertex e to vertex e + 1 as A a + B b + C; at the third
        // vertex every edge function equals twice the signed area, so with
        // all three negated for a negative area the interior is e >= 0 on
        // every edge (negation is exact before and after rounding)
        double vy[3], vz[3];
        for (int i = 0; i < 3; ++i) {
          vy[i] = (v[2 * i] - q.ymid) * ki;
          vz[i] = (v[2 * i + 1] - q.zmid) * ki;
        }
        const double area2 = (vy[1] - vy[0]) * (vz[2] - vz[0]) - (vz[1] - vz[0]) * (vy[2] - vy[0]);
        const double o = area2 < 0.0 ? -1.0 : 1.0;
        for (int e = 0; e < 3; ++e) {
          const int l = (e + 1) % 3;
          q.pf[k][3 * e] = (float)(o * -(vz[l] - vz[e]));
          q.pf[k][3 * e + 1] = (float)(o * (vy[l] - vy[e]));
          q.pf[k][3 * e + 2] = (float)(o * ((vz[l] - vz[e]) * vy[e] - (vy[l] - vy[e]) * vz[e]));
        }
      }
    }
  }
  q.c[np] = alpha_of(r, m, m.desc.sigma_background) * r.dt / 2.0;
  // model signature: air above z0 first, then at most one other primitive
  q.sig = kSigGeneric;
  const auto &R = m.regions;
  if (np == 0) {
    q.sig = kSigNone;
  } else if (R[0].kind == SDD_HALF_Z_LT && np <= 2) {
    q.sigp[0] = (float)((R[0].v[0] - q.zmid) * ki);
    if (np == 1) {
      q.sig = kSigZ;
    } else if (R[1].kind == SDD_HALF_Y_LT) {
      q.sig = kSigZY;
      q.sigp[1] = (float)((R[1].v[0] - q.ymid) * ki);
    } else if (R[1].kind == SDD_BOX) {
      q.sig = kSigZBox;
      q.sigp[1] = (float)((R[1].v[0] - q.ymid) * ki);
      q.sigp[2] = (float)((R[1].v[1] - q.ymid) * ki);
      q.sigp[3] = (float)((R[1].v[2] - q.zmid) * ki);
      q.sigp[4] = (float)((R[1].v[3] - q.zmid) * ki);
    } else if (R[1].kind == SDD_TRIANGLE) {
      q.sig = kSigZTri;
      // the three oriented edges (A, B, C) of the primitive's FP32 geometry
      for (int i = 0; i < 9; ++i) q.sigp[1 + i] = q.pf[1][i];
    }
  }
  q.fhy = (float)(0.5 * (q.y_hi - q.y_lo) * ki);
  q.fhz = (float)(0.5 * (q.z_hi - q.z_lo) * ki);
  // FP32 uniforms are at least 2^-24, so -log2(U) / 2 <= 12: no bridge hit is
  // possible once 2 d0 d1 > 12.05 (16.7 dt in unscaled lengths)
  q.fthr = 12.05f;
  q.fscr = 0.5f * q.fthr;
  // naive exits: no bridge test (2 d0 d1 > 0 always exceeds a negative
  // threshold), crossings only; the screens still flag every crossing
  if (r.flags & SDD_FLAG_EXIT_NAIVE) {
    q.thr = -1.0;
    q.fthr = -1.0f;
  }
  q.fscr_root = sqrtf(q.fscr);
  while (!(q.fscr_root * q.fscr_root > q.fscr)) q.fscr_root = nextafterf(q.fscr_root, INFINITY);
  // fixed-point phase increments of the generic FP32 walk: the largest one in
  // [2^29, 2^30] (bit 31 is the sigma grid's loop mark), so a 64-bit sum holds
  // 2^32 steps exactly
  {
    double cmax = 0.0;
    for (uint32_t k = 0; k <= np; ++k) cmax = std::max(cmax, q.c[k]);
    int e = 0;
    if (cmax > 0.0) (void)std::frexp(cmax, &e);
    q.phase_shift = cmax > 0.0 ? 30 - e : 0;
    for (uint32_t k = 0; k <= np; ++k) q.cfx[k] = (uint32_t)std::llround(std::ldexp(q.c[k], q.phase_shift));
  }
  q.key0 = (uint32_t)(r.seed & 0xFFFFFFFFu);
  q.key1 = (uint32_t)(r.seed >> 32);
  q.ctr3 = 2u * r.stream;
  q.max_steps = r.max_steps ? r.max_steps : kDefaultMaxSteps;
  q.cap2 = q.max_steps >= 2u ? q.max_steps - 2u : 0u;
  q.cap2b = q.cap2 >= 2u ? q.cap2 - 2u : 0u;
  q.cap_odd = q.max_steps & 1u;
  q.precision = (uint32_t)r.precision;
  q.M = r.g_samples - 1;
  q.model = reinterpret_cast<const DevModel *>(m.dev);
  P.grid.clear();
  P.grid_ext.clear();
  P.lds.clear();
  q.grid = nullptr;
  q.grid_ext = nullptr;
  q.lds_src = nullptr;
  q.lds_bytes = q.lds_table = 0;
  if (q.sig == kSigGeneric && r.precision == SDD_FP32_MIXED && !(r.flags & SDD_FLAG_NO_SIGMA_GRID) && np > 0) {
    build_sigma_grid(q, P.grid, P.grid_ext);
    if (!(r.flags & SDD_FLAG_NO_LDS_GRID))
      build_lds_form(P.grid, P.grid_ext, P.owner->lds_per_block, P.lds, q.lds_table);
    q.lds_bytes = (uint32_t)P.lds.size();
  }
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

// Waves of a typical launch: 4 SIMDs per CU, 4 waves each.
static uint64_t launch_waves_estimate(sdd_ctx *ctx) { return (uint64_t)std::max(ctx->cus, 1) * 4 * 4; }

// Expected exit time of standard Brownian motion from the rectangle, up to a
// factor below 2: the harmonic mean of the two 1-D exit times (y - y_lo)
// (y_hi - y) and (z - z_lo)(z_hi - z).  Used only to order work.
static double exit_time_estimate(const DevReq &q, double y, double z) {
  const double a = (y - q.y_lo) * (q.y_hi - y), b = (z - q.z_lo) * (q.z_hi - z);
  return (a > 0.0 && b > 0.0) ? a * b / (a + b) : 0.0;
}

// Paths per tile near the end of a request's work: the share of the paths
// still unclaimed that keeps every wave of a launch (about `waves` of them)
// busy, down to one path per lane, so the waves run out of work together
// instead of a few of them finishing whole tiles alone.
static uint32_t guided_tile(uint64_t remaining, uint64_t waves, uint32_t cap) {
  uint64_t want = remaining / (2 * std::max<uint64_t>(waves, 1));
  want = std::max<uint64_t>(want / 64 * 64, 64);
  return (uint32_t)std::min<uint64_t>(want, std::max<uint32_t>(cap, 1u));
}

// Tiles of each node's paths (record slots node-major in path order), in the
// order waves claim them: nodes with the longest expected paths first, so the
// last tiles of a launch hold short paths, and tile sizes shrink (guided) as
// the request's paths run out.  Results do not depend on the order or sizes.
static void build_tiles(Prepared &P, uint32_t cap, uint64_t waves) {
  const uint32_t n = (uint32_t)P.pbeg.size();
  P.tiles.clear();
  P.rec_off.assign(n + 1, 0);
  uint64_t off = 0;
  for (uint32_t j = 0; j < n; ++j) {
    P.rec_off[j] = off;
    off += P.pcnt[j];
  }
  P.rec_off[n] = off;
  P.n_paths = off;
  std::vector<uint32_t> order(n);
  std::vector<double> key(n);
  for (uint32_t j = 0; j < n; ++j) {
    order[j] = j;
    key[j] = exit_time_estimate(P.dreq, P.nodes[2 * j], P.nodes[2 * j + 1]);
  }
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return key[a] > key[b]; });
  uint64_t remaining = off;
  for (uint32_t j : order) {
    const uint32_t b = P.pbeg[j], c = P.pcnt[j];
    uint32_t k = 0;
    while (k < c) {
      const uint32_t cnt = std::min(guided_tile(remaining, waves, cap), c - k);
      DevTile t{};
      t.node = j;
      t.p0 = b + k;
      t.count = cnt;
      t.rec0 = P.rec_off[j] + k;
      P.tiles.push_back(t);
      k += cnt;
      remaining -= cnt;
    }
  }
}

// Largest paths per tile: the tuned size, lowered for a small request so that
// its tiles reach every wave of a launch instead of queueing behind a few.
static uint32_t tile_size(sdd_ctx *ctx, const Prepared &P) {
  const uint32_t cap = ctx->tuning.tile_paths ? ctx->tuning.tile_paths : 512u;
  uint64_t total = 0;
  for (uint32_t c : P.pcnt) total += c;
  const uint64_t waves = launch_waves_estimate(ctx);
  const uint64_t per = ((total + waves - 1) / waves + 63) / 64 * 64;
  return (uint32_t)std::min<uint64_t>(cap, std::max<uint64_t>(per, 64));
}

static size_t pass_bytes(const Prepared &P) {
  return Arena::round(P.g.size() * 8) + Arena::round(P.nodes.size() * 8 + 16) +
         Arena::round(P.grid.size() * sizeof(SigmaCell)) + Arena::round(P.grid_ext.size() * sizeof(SigmaCell)) +
         Arena::round(P.lds.size()) +
         Arena::round(P.tiles.size() * sizeof(DevTile) + 16) + Arena::round(P.n_paths * sizeof(PathRec) + 16);
}

static void release_pass(sdd_ctx *ctx, Prepared &P) {
  ctx->release(P.d_g);
  ctx->release(P.d_nodes);
  ctx->release(P.d_tiles);
  ctx->release(P.d_recs);
  ctx->release(P.d_grid);
  ctx->release(P.d_grid_ext);
  ctx->release(P.d_lds);
  P.d_g = P.d_nodes = P.d_tiles = P.d_recs = P.d_grid = P.d_grid_ext = P.d_lds = nullptr;
}

static void release_all(sdd_ctx *ctx, Prepared &P) {
  release_pass(ctx, P);
  ctx->release(P.d_recs_pilot);
  P.d_recs_pilot = nullptr;
}

// Allocate and upload one pass's inputs (caller holds ctx->mu).
static sdd_status upload_pass(sdd_ctx *ctx, Prepared &P) {
  build_tiles(P, tile_size(ctx, P), launch_waves_estimate(ctx));
  P.d_g = ctx->alloc(P.g.size() * 8);
  P.d_nodes = ctx->alloc(P.nodes.size() * 8 + 16);
  P.d_tiles = ctx->alloc(P.tiles.size() * sizeof(DevTile) + 16);
  P.d_recs = ctx->alloc(P.n_paths * sizeof(PathRec) + 16);
  if (!P.grid.empty()) P.d_grid = ctx->alloc(P.grid.size() * sizeof(SigmaCell));
  if (!P.lds.empty()) P.d_lds = ctx->alloc(P.lds.size());
  if (!P.grid_ext.empty()) P.d_grid_ext = ctx->alloc(P.grid_ext.size() * sizeof(SigmaCell));
  if (!P.d_g || !P.d_nodes || !P.d_tiles || !P.d_recs || (!P.grid.empty() && !P.d_grid) ||
      (!P.lds.empty() && !P.d_lds) || (!P.grid_ext.empty() && !P.d_grid_ext)) {
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
  P.dreq.grid = nullptr;
  if (!P.grid.empty()) {
    HIP_TRY(hipMemcpyAsync(P.d_grid, P.grid.data(), P.grid.size() * sizeof(SigmaCell), hipMemcpyHostToDevice,
                           ctx->stream));
    P.dreq.grid = reinterpret_cast<const SigmaCell *>(P.d_grid);
  }
  P.dreq.grid_ext = nullptr;
  if (!P.grid_ext.empty()) {
    HIP_TRY(hipMemcpyAsync(P.d_grid_ext, P.grid_ext.data(), P.grid_ext.size() * sizeof(SigmaCell),
                           hipMemcpyHostToDevice, ctx->stream));
    P.dreq.grid_ext = reinterpret_cast<const SigmaCell *>(P.d_grid_ext);
  }
  P.dreq.lds_src = nullptr;
  if (!P.lds.empty()) {
    HIP_TRY(hipMemcpyAsync(P.d_lds, P.lds.data(), P.lds.size(), hipMemcpyHostToDevice, ctx->stream));
    P.dreq.lds_src = reinterpret_cast<const uint8_t *>(P.d_lds);
  }
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

static uint32_t refill_mask(const sdd_ctx *ctx) {
  return ctx->tuning.refill_every ? ctx->tuning.refill_every - 1u : 0u;
}

// The model signature shared by every request of a launch, or -1 if they
// differ (then the walker that handles every signature is launched).
template <class It, class Get>
static int common_sig(It begin, It end, Get get) {
  int sig = -2;
  for (It i = begin; i != end; ++i) {
    const int s = get(*i);
    if (sig == -2) sig = s;
    else if (sig != s) return -1;
  }
  return sig == -2 ? -1 : sig;
}

// The walker build of a launch over passes of one precision: the model
// signature every pass shares (or -1), turned into kSigGenericLds when every
// pass is an FP32-mixed generic request with the same sigma grid (the same
// model, time step and frequency: identical LDS forms and cell mapping); then
// lds_bytes is the size of that form.
static bool same_lds_grid(const Prepared &a, const Prepared &b) {
  const DevReq &x = a.dreq, &y = b.dreq;
  return a.lds == b.lds && x.lds_table == y.lds_table && x.gy == y.gy && x.gz == y.gz && x.gsy == y.gsy &&
         x.goy == y.goy && x.gsz == y.gsz && x.goz == y.goz;
}

template <class It, class Get>
static int launch_sig(It begin, It end, Get get, uint32_t &lds_bytes) {
  lds_bytes = 0;
  const int sig = common_sig(begin, end, [&](const auto &x) { return get(x)->dreq.sig; });
  if (sig != kSigGeneric) return sig;
  const Prepared *first = get(*begin);
  if (first->dreq.precision != SDD_FP32_MIXED || first->lds.empty()) return sig;
  for (It i = begin; i != end; ++i)
    if (!same_lds_grid(*first, *get(*i))) return sig;
  lds_bytes = (uint32_t)first->lds.size();
  return kSigGenericLds;
}

static void launch_shape(sdd_ctx *ctx, int precision, int sig, uint32_t lds_bytes, uint32_t &blocks,
                         uint32_t &threads) {
  if (sig == kSigGenericLds) {   // its own block size; the tuned block shape is for the others
    threads = lds_walker_threads();
    const int occ = persist_blocks_per_cu(precision, sig, threads, lds_bytes);
    blocks = (uint32_t)ctx->cus * (occ > 0 ? (uint32_t)occ : 1u);
    return;
  }
  threads = ctx->tuning.block_threads ? ctx->tuning.block_threads : 256u;
  uint32_t per_cu = ctx->tuning.blocks_per_cu;
  if (!per_cu) {
    const int occ = persist_blocks_per_cu(precision, sig, threads, 0);
    per_cu = occ > 0 ? (uint32_t)occ : 1u;
  }
  blocks = (uint32_t)ctx->cus * per_cu;
}

// One persistent launch over passes of one precision (the walker kernel is
// compiled per precision).
static sdd_status run_group(sdd_ctx *ctx, std::vector<Prepared *> &passes, int precision) {
  const uint32_t n = (uint32_t)passes.size();
  if (n == 0) return SDD_OK;
  uint32_t blocks, threads, lds_bytes;
  const int sig = launch_sig(passes.begin(), passes.end(), [](const Prepared *P) { return P; }, lds_bytes);
  launch_shape(ctx, precision, sig, lds_bytes, blocks, threads);
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
    if (sig == kSigGenericLds) dq[i].sig = kSigGenericLds;
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
    check(launch_walk_persist(precision, sig, reinterpret_cast<const DevReq *>(B.d_reqs), n,
                              reinterpret_cast<const uint32_t *>(B.d_ws), 0u, refill_mask(ctx), blocks, threads,
                              lds_bytes, ctx->stream),
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

// |g|inf of a request's tables (interleaved re, im).
static double g_norm(const std::vector<double> &g) {
  double m = 0.0;
  for (size_t k = 0; k + 1 < g.size(); k += 2) m = std::max(m, std::hypot(g[k], g[k + 1]));
  return m;
}

// After a pilot pass: decide each node's path count and set up the extension.
static void plan_extension(Prepared &P, const NodeOut *pilot_rows) {
  const uint32_t n = (uint32_t)P.pbeg_all.size();
  const double gnorm = g_norm(P.g);
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

static void scatter_rows(uint32_t n, const NodeOut *rows, sdd_result *res) {
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

// The diagnostics block of a result: rho_dt, its flag, |g|inf and the
// largest se / |g|inf over the nodes.
static void fill_diag(sdd_diag *d, double rho_dt, double gn, uint32_t n, const NodeOut *rows) {
  if (!d) return;
  std::memset(d, 0, sizeof(*d));
  d->rho_dt = rho_dt;
  d->flags = rho_dt > 0.1 ? SDD_DIAG_DT_UNRESOLVED : 0u;
  d->g_norm = gn;
  double se = 0.0;
  for (uint32_t j = 0; j < n; ++j)
    if (std::isfinite(rows[j].se)) se = std::max(se, rows[j].se);
  d->se_over_gnorm = gn > 0.0 ? se / gn : 0.0;
}

static void scatter(const Prepared &P, const NodeOut *rows, sdd_result *res) {
  const uint32_t n = (uint32_t)P.pbeg_all.size();
  scatter_rows(n, rows, res);
  double rho = 0.0;
  for (uint32_t k = 0; k <= P.dreq.nprims; ++k) rho = std::max(rho, P.dreq.c[k]);
  fill_diag(res->diag, rho, g_norm(P.g), n, rows);
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

// Workspace a request's current pass needs while it runs: tables, nodes,
// sigma grid, tiles, records, the reduction and the launch descriptors.  A
// target-SE request's first pass is its pilot; with `upper`, its extension
// at the largest size (2^20 paths per node) is added: the bound for a
// blocking solve, which keeps the pilot's records while it walks the
// extension.
static uint64_t footprint(sdd_ctx *ctx, Prepared &P, bool upper) {
  build_tiles(P, tile_size(ctx, P), launch_waves_estimate(ctx));
  const uint64_t n = P.pbeg.size();
  uint64_t b = pass_bytes(P) + Arena::round(n * (sizeof(NodeOut) + sizeof(NodeJob))) + 4 * 1024 +
               Arena::round(sizeof(DevReq) * 2);
  if (upper && P.req.target_rel_se > 0.0 && P.pass == 0)
    b += Arena::round(n * (uint64_t)kMaxTargetPaths * sizeof(PathRec));
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

// A request in flight in served mode: its passes run in time slices of the
// persistent walker; at each slice end the walkers still running are
// suspended into `pool` and partly used tiles into `extra`, double-buffered
// (index `par` is what the next slice resumes from).
struct Flight {
  std::shared_ptr<Ticket> T;
  Prepared *P = nullptr;
  bool uploaded = false;
  char *d_pool[2] = {nullptr, nullptr}, *d_extra[2] = {nullptr, nullptr};
  uint32_t pool_cap = 0, extra_cap = 0;
  int par = 0;
  uint32_t pool_n = 0, extra_n = 0;
  uint32_t tile_counter = 0;
  uint64_t done = 0;
  uint64_t reserved = 0;   // workspace bytes promised to this flight
  bool requeue = false;    // give the workspace back and wait for admission again
};

// Suspension pools of a served flight at the launch shape of its own walker
// build: two buffers of suspended walkers (each up to two per lane: the
// slice's own and those a narrower launch left) and two of tile remainders
// (two per wave).
static uint64_t pool_bytes(sdd_ctx *ctx, const Prepared &P) {
  uint32_t blocks, threads;
  launch_shape(ctx, (int)P.dreq.precision, P.dreq.sig, 0, blocks, threads);
  const uint64_t lanes = (uint64_t)blocks * threads, waves = lanes / 64;
  return 2 * Arena::round(2 * lanes * sizeof(SuspRec)) + 2 * Arena::round(2 * waves * sizeof(DevTile));
}

// Control words of one flight for one slice (device and host copies).
struct FlightCtl {
  uint32_t slice[4];
  uint32_t tile_counter;
  uint32_t pad;
  unsigned long long done;
};

static void release_flight(sdd_ctx *ctx, Flight &F) {
  for (int i = 0; i < 2; ++i) {
    ctx->release(F.d_pool[i]);
    ctx->release(F.d_extra[i]);
    F.d_pool[i] = F.d_extra[i] = nullptr;
  }
  if (F.P) release_all(ctx, *F.P);
}

// Pools for one slice: its output must hold every walker the launch can
// suspend (one per lane) and every tile remainder (one per wave), plus the
// entries of the input pools that the slice leaves unclaimed (carried over by
// the host; a launch may have fewer lanes than the previous slice had).
// Suspended walkers already waiting in the input pool are kept.
// The first pools hold two per lane and per wave (what the flight's
// reservation counts), so slices at one launch shape never reallocate them.
static sdd_status ensure_pools(sdd_ctx *ctx, Flight &F, uint32_t lanes, uint32_t waves) {
  const uint32_t need_p = lanes + F.pool_n, need_e = waves + F.extra_n;
  if (F.pool_cap >= need_p && F.extra_cap >= need_e && F.d_pool[0]) return SDD_OK;
  const uint32_t cap_p = std::max({need_p, F.pool_cap, 2 * lanes}), cap_e = std::max({need_e, F.extra_cap, 2 * waves});
  char *np[2] = {ctx->alloc((size_t)cap_p * sizeof(SuspRec)), ctx->alloc((size_t)cap_p * sizeof(SuspRec))};
  char *ne[2] = {ctx->alloc((size_t)cap_e * sizeof(DevTile)), ctx->alloc((size_t)cap_e * sizeof(DevTile))};
  if (!np[0] || !np[1] || !ne[0] || !ne[1]) {
    for (int i = 0; i < 2; ++i) { ctx->release(np[i]); ctx->release(ne[i]); }
    return fail(SDD_E_NOMEM, "no workspace left for the suspension pools");
  }
  if (F.pool_n) HIP_TRY(hipMemcpyAsync(np[F.par], F.d_pool[F.par], (size_t)F.pool_n * sizeof(SuspRec),
                                       hipMemcpyDeviceToDevice, ctx->stream));
  if (F.extra_n) HIP_TRY(hipMemcpyAsync(ne[F.par], F.d_extra[F.par], (size_t)F.extra_n * sizeof(DevTile),
                                        hipMemcpyDeviceToDevice, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < 2; ++i) {
    ctx->release(F.d_pool[i]);
    ctx->release(F.d_extra[i]);
    F.d_pool[i] = np[i];
    F.d_extra[i] = ne[i];
  }
  F.pool_cap = cap_p;
  F.extra_cap = cap_e;
  return SDD_OK;
}

// One time slice over the flights of one precision (caller holds exec).
static sdd_status run_slice(sdd_ctx *ctx, std::vector<Flight *> &fl, int precision) {
  const uint32_t n = (uint32_t)fl.size();
  if (n == 0) return SDD_OK;
  uint32_t blocks, threads, lds_bytes;
  const int sig = launch_sig(fl.begin(), fl.end(), [](const Flight *F) { return F->P; }, lds_bytes);
  launch_shape(ctx, precision, sig, lds_bytes, blocks, threads);
  const uint32_t lanes = blocks * threads, waves = blocks * (threads / 64);
  for (auto *F : fl) {
    sdd_status st = ensure_pools(ctx, *F, lanes, waves);
    if (st != SDD_OK) return st;
  }
  char *d_reqs = ctx->alloc(n * sizeof(DevReq));
  char *d_ctl = ctx->alloc(n * sizeof(FlightCtl));
  char *d_ws = ctx->alloc((n + 1) * sizeof(uint32_t));
  sdd_status st = SDD_OK;
  if (!d_reqs || !d_ctl || !d_ws) st = fail(SDD_E_NOMEM, "no workspace left for a slice");
  std::vector<DevReq> dq(n);
  std::vector<FlightCtl> ctl(n);
  std::vector<uint32_t> ws(n + 1, 0);
  // Wave shares, shortest remaining work first: every flight holds at least
  // waves / 4n waves, then flights in order of remaining paths get the waves
  // that cover them.  Waves left over start on whichever flight has the most
  // work left, as do waves whose flight runs dry.
  std::vector<uint64_t> rem(n), share(n);
  std::vector<uint32_t> order(n);
  const uint64_t floor_w = std::max<uint64_t>(1, waves / (4ull * n));
  uint64_t given = 0;
  for (uint32_t i = 0; i < n; ++i) {
    rem[i] = fl[i]->P->n_paths - std::min<uint64_t>(fl[i]->done, fl[i]->P->n_paths);
    share[i] = std::min<uint64_t>({(rem[i] + 63) / 64, floor_w, waves - given});
    given += share[i];
    order[i] = i;
  }
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return rem[a] < rem[b]; });
  for (uint32_t i : order) {
    const uint64_t add = std::min<uint64_t>((rem[i] + 63) / 64 - share[i], waves - given);
    share[i] += add;
    given += add;
  }
  uint64_t acc = 0;
  for (uint32_t i = 0; i < n && st == SDD_OK; ++i) {
    Flight &F = *fl[i];
    FlightCtl &c = ctl[i];
    std::memset(&c, 0, sizeof(c));
    c.tile_counter = F.tile_counter;
    c.done = F.done;
    FlightCtl *dc = reinterpret_cast<FlightCtl *>(d_ctl) + i;
    DevReq &q = dq[i];
    q = F.P->dreq;
    if (sig == kSigGenericLds) q.sig = kSigGenericLds;
    q.tile_counter = &dc->tile_counter;
    q.done_counter = &dc->done;
    q.slice_ctl = dc->slice;
    q.pool_in = reinterpret_cast<const SuspRec *>(F.d_pool[F.par]);
    q.pool_in_n = F.pool_n;
    q.pool_out = reinterpret_cast<SuspRec *>(F.d_pool[F.par ^ 1]);
    q.pool_cap = F.pool_cap;
    q.extra_in = reinterpret_cast<const DevTile *>(F.d_extra[F.par]);
    q.extra_in_n = F.extra_n;
    q.extra_out = reinterpret_cast<DevTile *>(F.d_extra[F.par ^ 1]);
    q.extra_cap = F.extra_cap;
    ws[i] = (uint32_t)acc;
    acc += share[i];
  }
  ws[n] = (uint32_t)acc;
  hipError_t e = hipSuccess;
  if (st == SDD_OK) {
    e = hipMemcpyAsync(d_reqs, dq.data(), n * sizeof(DevReq), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_ctl, ctl.data(), n * sizeof(FlightCtl), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_ws, ws.data(), (n + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipEventRecord(ctx->ev[0], ctx->stream);
    if (e == hipSuccess)
      e = launch_walk_persist(precision, sig, reinterpret_cast<const DevReq *>(d_reqs), n,
                              reinterpret_cast<const uint32_t *>(d_ws),
                              ctx->tuning.slice_iters ? ctx->tuning.slice_iters : 4096u, refill_mask(ctx), blocks, threads,
                              lds_bytes, ctx->stream);
    if (e == hipSuccess) e = hipEventRecord(ctx->ev[1], ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ctl.data(), d_ctl, n * sizeof(FlightCtl), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) st = fail(SDD_E_DEVICE, "slice: %s", hipGetErrorString(e));
  }
  ctx->release(d_reqs);
  ctx->release(d_ctl);
  ctx->release(d_ws);
  if (st != SDD_OK) return st;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]) == hipSuccess) ctx->stats.last_walk_ms = ms;
  ctx->stats.launches += 1;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->served_walk_ms += ms;
    ctx->served_slices += 1;
  }
  for (uint32_t i = 0; i < n; ++i) {
    Flight &F = *fl[i];
    const FlightCtl &c = ctl[i];
    // entries of the input pools no wave claimed move to the end of the
    // output pools
    const uint32_t pc = std::min(c.slice[kPoolCursor], F.pool_n);
    const uint32_t ec = std::min(c.slice[kExtraCursor], F.extra_n);
    const uint32_t carry_p = F.pool_n - pc, carry_e = F.extra_n - ec;
    if (c.slice[kPoolOut] + carry_p > F.pool_cap || c.slice[kExtraOut] + carry_e > F.extra_cap)
      return fail(SDD_E_DEVICE, "suspension pool overflow (%u + %u > %u walkers)", c.slice[kPoolOut], carry_p,
                  F.pool_cap);
    const int in = F.par, out = F.par ^ 1;
    if (carry_p)
      HIP_TRY(hipMemcpyAsync(F.d_pool[out] + (size_t)c.slice[kPoolOut] * sizeof(SuspRec),
                             F.d_pool[in] + (size_t)pc * sizeof(SuspRec), (size_t)carry_p * sizeof(SuspRec),
                             hipMemcpyDeviceToDevice, ctx->stream));
    if (carry_e)
      HIP_TRY(hipMemcpyAsync(F.d_extra[out] + (size_t)c.slice[kExtraOut] * sizeof(DevTile),
                             F.d_extra[in] + (size_t)ec * sizeof(DevTile), (size_t)carry_e * sizeof(DevTile),
                             hipMemcpyDeviceToDevice, ctx->stream));
    F.par = out;
    F.pool_n = c.slice[kPoolOut] + carry_p;
    F.extra_n = c.slice[kExtraOut] + carry_e;
    // claims past the last tile (waves racing for it) carry no work: the next
    // slice starts from n_tiles at most, so the counter never wraps
    F.tile_counter = std::min(c.tile_counter, F.P->dreq.n_tiles);
    F.done = c.done;
  }
  return SDD_OK;
}

// Hands a flight's workspace back: its passes, its pools and its reservation.
static void drop_flight(sdd_ctx *ctx, Flight &F) {
  release_flight(ctx, F);
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->reserved -= std::min(ctx->reserved, F.reserved);
  F.reserved = 0;
}

// After a target-SE pilot: reduce it, plan each node's path count and set up
// the extension.  The extension gets the workspace it needs if that fits
// next to the other flights' reservations; otherwise the flight gives all of
// its workspace back (pilot records included) and is re-queued to walk every
// path of every node in one pass once admitted again -- the same paths, read
// by the reduction in the same order, so the result is the same bit for bit.
static sdd_status start_extension(sdd_ctx *ctx, Flight &F) {
  Prepared &P = *F.P;
  std::vector<Prepared *> one{&P};
  std::vector<NodeOut> rows;
  sdd_status st = reduce_passes(ctx, one, rows);
  if (st != SDD_OK) return st;
  plan_extension(P, rows.data());
  P.d_recs_pilot = P.d_recs;
  P.d_recs = nullptr;
  release_pass(ctx, P);
  const uint64_t pilot_recs = Arena::round(P.n_paths * sizeof(PathRec) + 16);
  const uint64_t need = footprint(ctx, P, false) + pilot_recs + pool_bytes(ctx, P);
  bool fits;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    const uint64_t cap = ctx->arena.size() > ctx->held_long ? ctx->arena.size() - ctx->held_long : 0;
    fits = ctx->reserved - F.reserved + need <= cap;
    if (fits && need > F.reserved) {
      ctx->reserved += need - F.reserved;
      F.reserved = need;
    }
  }
  if (ctx->debug)
    std::fprintf(stderr, "[sdd] extension needs %llu (reserved %llu): %s\n", (unsigned long long)need,
                 (unsigned long long)F.reserved, fits ? "fits" : "re-queued");
  st = fits ? upload_pass(ctx, P) : SDD_E_NOMEM;
  if (st == SDD_OK) {
    F.uploaded = true;
    F.tile_counter = 0;
    F.done = 0;
    F.pool_n = F.extra_n = 0;
    return SDD_OK;
  }
  if (st != SDD_E_NOMEM) return st;
  ctx->release(P.d_recs_pilot);
  P.d_recs_pilot = nullptr;
  P.pbeg = P.pbeg_all;
  P.pcnt = P.pcnt_all;
  P.pass = 2;
  F.requeue = true;
  return SDD_OK;
}

// Moves the flights marked for re-queueing back to the front of the
// admission order (in their order), their workspace given back.
static void requeue_flights(sdd_ctx *ctx, std::vector<std::unique_ptr<Flight>> &flights) {
  std::vector<std::shared_ptr<Ticket>> back;
  for (auto &F : flights) {
    if (!F->requeue) continue;
    drop_flight(ctx, *F);
    back.push_back(F->T);
    F->P = nullptr;
  }
  if (back.empty()) return;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (auto &T : back) ctx->served_requeues += T->P && T->P->pass == 2 ? 1u : 0u;
  }
  flights.erase(std::remove_if(flights.begin(), flights.end(), [](const std::unique_ptr<Flight> &F) { return F->P == nullptr; }),
                flights.end());
  std::lock_guard<std::mutex> lk(ctx->mu);
  for (auto it = back.rbegin(); it != back.rend(); ++it) ctx->requeue.push_front(*it);
}

// Finish the flights whose pass has every path done: a pilot is turned into
// its extension; everything else is reduced and handed back.
static void complete_flights(sdd_ctx *ctx, std::vector<std::unique_ptr<Flight>> &flights) {
  std::vector<Flight *> fin;
  for (auto &F : flights) {
    if (F->requeue || F->done < F->P->n_paths || F->pool_n || F->extra_n) continue;
    if (F->P->req.target_rel_se > 0.0 && F->P->pass == 0 && F->T->status == SDD_OK) {
      const sdd_status st = start_extension(ctx, *F);
      if (st == SDD_OK) continue;
      F->T->error = g_last_error;
      F->T->status = st;
    }
    fin.push_back(F.get());
  }
  requeue_flights(ctx, flights);
  if (fin.empty()) return;
  std::vector<Prepared *> Ps;
  for (auto *F : fin)
    if (F->T->status == SDD_OK) Ps.push_back(F->P);
  std::vector<NodeOut> rows;
  sdd_status st = reduce_passes(ctx, Ps, rows);
  std::string err = st == SDD_OK ? std::string() : g_last_error;
  uint64_t row = 0;
  for (auto *P : Ps) {
    Flight *F = nullptr;
    for (auto *f : fin)
      if (f->P == P) F = f;
    if (st == SDD_OK && !F->T->cancelled) {
      scatter(*P, rows.data() + row, &F->T->res);
      sdd_status s2 = copy_records(ctx, *P, &F->T->res);
      if (s2 != SDD_OK) { F->T->status = s2; F->T->error = g_last_error; }
    } else if (st != SDD_OK) {
      F->T->status = st;
      F->T->error = err;
    }
    row += P->pbeg.size();
  }
  for (auto *F : fin) drop_flight(ctx, *F);
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (auto *F : fin) {
      finish_ticket(ctx, *F->T, F->T->status, F->T->error.empty() ? nullptr : F->T->error.c_str());
      F->T->P.reset();
      F->P = nullptr;
    }
  }
  flights.erase(std::remove_if(flights.begin(), flights.end(), [](const std::unique_ptr<Flight> &F) { return F->P == nullptr; }),
                flights.end());
  ctx->done_cv.notify_all();
}

// Admission (caller holds ctx->mu): re-queued flights first, then the queue,
// each in order, while the promised footprints fit in the workspace less
// what models and prepared batches hold.  A request that could not fit even
// in that much is failed with SDD_E_NOMEM; one that only has to wait for
// memory keeps its place and everything behind it waits too.
static void admit(sdd_ctx *ctx, std::vector<std::unique_ptr<Flight>> &flights) {
  const uint64_t cap = ctx->arena.size() > ctx->held_long ? ctx->arena.size() - ctx->held_long : 0;
  for (auto *q : {&ctx->requeue, &ctx->queue}) {
    while (!q->empty()) {
      auto T = q->front();
      const uint64_t need = footprint(ctx, *T->P, false) + pool_bytes(ctx, *T->P);
      if (need > cap) {
        q->pop_front();
        char msg[192];
        std::snprintf(msg, sizeof(msg),
                      "request needs %llu bytes of workspace; %llu are left beside the resident models and "
                      "prepared batches",
                      (unsigned long long)need, (unsigned long long)cap);
        finish_ticket(ctx, *T, SDD_E_NOMEM, msg);
        T->P.reset();
        ctx->done_cv.notify_all();
        continue;
      }
      if (ctx->reserved + need > cap) {   // wait for memory to free up
        if (!T->waited) {
          T->waited = true;
          ++ctx->served_waits;
        }
        if (ctx->debug)
          std::fprintf(stderr, "[sdd] admission waits: needs %llu, %llu of %llu promised\n",
                       (unsigned long long)need, (unsigned long long)ctx->reserved, (unsigned long long)cap);
        return;
      }
      auto F = std::make_unique<Flight>();
      F->T = T;
      F->P = T->P.get();
      F->reserved = need;
      ctx->reserved += need;
      if (ctx->debug)
        std::fprintf(stderr, "[sdd] admitted (%s): reserves %llu, %llu of %llu promised\n",
                     q == &ctx->requeue ? "again, one pass" : "new", (unsigned long long)need,
                     (unsigned long long)ctx->reserved, (unsigned long long)cap);
      flights.push_back(std::move(F));
      q->pop_front();
      ctx->served_in_flight_max = std::max(ctx->served_in_flight_max, (uint32_t)flights.size());
    }
  }
}

static void worker_main(sdd_ctx *ctx) {
  // if this fails, the worker's first HIP call fails too and its tickets
  // report SDD_E_DEVICE
  (void)hipSetDevice(ctx->device);
  std::vector<std::unique_ptr<Flight>> flights;
  // memory epoch at which admission last stalled with nothing in flight: the
  // worker then sleeps until memory is released or the queue changes
  uint64_t stalled_at = ~0ull;
  for (;;) {
    std::vector<std::unique_ptr<Flight>> dropped;
    bool stop;
    {
      std::unique_lock<std::mutex> lk(ctx->mu);
      ctx->cv.wait(lk, [&] {
        return ctx->stop || !flights.empty() ||
               ((!ctx->queue.empty() || !ctx->requeue.empty()) && ctx->epoch != stalled_at);
      });
      stop = ctx->stop;
      if (stop) {
        for (auto *q : {&ctx->queue, &ctx->requeue}) {
          for (auto &T : *q) {
            T->cancelled = true;
            finish_ticket(ctx, *T, SDD_E_CANCELLED, "context destroyed");
            T->P.reset();
          }
          q->clear();
        }
        for (auto &F : flights) F->T->cancelled = true;
      }
      // cancelled flights leave at the slice boundary
      for (auto &F : flights)
        if (F->T->cancelled) dropped.push_back(std::move(F));
      flights.erase(std::remove(flights.begin(), flights.end(), nullptr), flights.end());
      if (!stop) admit(ctx, flights);
      if (flights.empty()) stalled_at = ctx->epoch;
    }
    for (auto &F : dropped) {
      auto ex = worker_exec(ctx);
      drop_flight(ctx, *F);
      std::lock_guard<std::mutex> lk(ctx->mu);
      finish_ticket(ctx, *F->T, SDD_E_CANCELLED, "cancelled");
      F->T->P.reset();
    }
    if (!dropped.empty()) ctx->done_cv.notify_all();
    if (stop && flights.empty()) return;
    if (flights.empty()) continue;
    {
      auto ex = worker_exec(ctx);
      // upload newly admitted requests.  While the worker holds exec, blocking
      // callers hold no workspace, so a request whose reservation fitted but
      // whose buffers do not (a fragmented workspace) waits for the running
      // flights to give theirs back, and fails if none is running.
      bool running = false;
      for (auto &F : flights) running = running || F->uploaded;
      for (auto &F : flights) {
        if (F->uploaded) continue;
        sdd_status st = upload_pass(ctx, *F->P);
        if (st == SDD_OK) {
          F->uploaded = true;
          running = true;
        } else if (st == SDD_E_NOMEM && running) {
          F->requeue = true;
        } else {
          F->T->status = st;
          F->T->error = g_last_error;
          F->done = F->P->n_paths;   // completes (with the error) below
          F->uploaded = true;
        }
      }
      requeue_flights(ctx, flights);
      // one slice per precision present
      for (int prec : {SDD_FP32_MIXED, SDD_FP64}) {
        std::vector<Flight *> group;
        for (auto &F : flights)
          if ((int)F->P->dreq.precision == prec && F->T->status == SDD_OK) group.push_back(F.get());
        const sdd_status st = run_slice(ctx, group, prec);
        if (st != SDD_OK) {
          for (auto *F : group) {
            F->T->status = st;
            F->T->error = g_last_error;
            F->done = F->P->n_paths;
            F->pool_n = F->extra_n = 0;
          }
        }
      }
      if (ctx->debug) {
        std::fprintf(stderr, "[sdd] slice %.3f ms:", ctx->stats.last_walk_ms);
        for (auto &F : flights)
          std::fprintf(stderr, " {done %llu/%llu tiles %u/%u pool %u extra %u}", (unsigned long long)F->done,
                       (unsigned long long)F->P->n_paths, F->tile_counter, F->P->dreq.n_tiles, F->pool_n,
                       F->extra_n);
        std::fprintf(stderr, "\n");
      }
      complete_flights(ctx, flights);
    }
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
  {
    void *sp = nullptr;
    HIP_TRY(scratch_init(device, &sp));
    ctx->scratch = reinterpret_cast<char *>(sp);
  }
  ctx->device = device;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  ctx->cus = prop.multiProcessorCount;
  ctx->lds_per_block = prop.sharedMemPerBlock;
  const char *dbg = std::getenv("SDD_DEBUG");
  ctx->debug = dbg && dbg[0] == '1';
  ctx->arena.init(reinterpret_cast<char *>(workspace_dev), workspace_bytes);
  *out = ctx.release();
  return SDD_OK;
}

sdd_status sdd_destroy(sdd_ctx_t ctx) {
  if (!ctx) return fail(SDD_E_INVALID, "ctx is NULL");
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->stop = true;
    ++ctx->epoch;
  }
  ctx->cv.notify_all();
  if (ctx->worker.joinable()) ctx->worker.join();
  {
    ExecGuard ex(ctx);   // no blocking call still running
    for (auto &e : ctx->ev)
      if (e) (void)hipEventDestroy(e);   // teardown: nothing to do on failure
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
    ExecGuard ex(ctx);
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
  ctx->held_long += Arena::round(sizeof(DevModel));
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
  ctx->held_long -= std::min<uint64_t>(ctx->held_long, Arena::round(sizeof(DevModel)));
  ++ctx->epoch;
  ctx->cv.notify_all();
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
  ExecGuard ex(ctx);
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

// H^x from the centred difference, less the first-order term of a jump of
// sigma between the outer points (zero inside one layer).
static sdd_status mt_te(uint32_t n, const double *e_minus, const double *e_mid, const double *e_plus, double h,
                        double length_unit_m, double freq_hz, double sigma_jump, double *rho_a, double *phase_deg) {
  if (n && (!e_minus || !e_mid || !e_plus || !rho_a || !phase_deg)) return fail(SDD_E_INVALID, "NULL array");
  if (!(h > 0.0) || !(length_unit_m > 0.0) || !(freq_hz > 0.0))
    return fail(SDD_E_INVALID, "h, length unit and frequency must be positive");
  if (!std::isfinite(sigma_jump)) return fail(SDD_E_INVALID, "sigma_jump must be finite");
  const double pi = 3.14159265358979323846;
  const double wmu = 2.0 * pi * freq_hz * (4e-7 * pi);
  const double hm = h * length_unit_m;
  const std::complex<double> kink(0.0, 0.25 * hm * wmu * sigma_jump);   // (h L / 4) i omega mu0 sigma_jump
  for (uint32_t j = 0; j < n; ++j) {
    const std::complex<double> em(e_minus[2 * j], e_minus[2 * j + 1]);
    const std::complex<double> e0(e_mid[2 * j], e_mid[2 * j + 1]);
    const std::complex<double> ep(e_plus[2 * j], e_plus[2 * j + 1]);
    std::complex<double> dedz = (ep - em) / (2.0 * hm);   // per metre
    if (sigma_jump != 0.0) dedz -= kink * e0;
    const std::complex<double> hx = -dedz / std::complex<double>(0.0, wmu);
    if (hx == std::complex<double>(0.0, 0.0)) {
      rho_a[j] = HUGE_VAL;
      phase_deg[j] = NAN;
      continue;
    }
    const std::complex<double> z = e0 / hx;
    rho_a[j] = std::norm(z) / wmu;
    phase_deg[j] = std::arg(z) * (180.0 / pi);
  }
  return SDD_OK;
}

sdd_status sdd_mt_te_response(uint32_t n, const double *e_minus, const double *e_mid, const double *e_plus, double h,
                              double length_unit_m, double freq_hz, double *rho_a, double *phase_deg) {
  return mt_te(n, e_minus, e_mid, e_plus, h, length_unit_m, freq_hz, 0.0, rho_a, phase_deg);
}

sdd_status sdd_mt_te_response_jump(uint32_t n, const double *e_minus, const double *e_mid, const double *e_plus,
                                   double h, double length_unit_m, double freq_hz, double sigma_jump, double *rho_a,
                                   double *phase_deg) {
  return mt_te(n, e_minus, e_mid, e_plus, h, length_unit_m, freq_hz, sigma_jump, rho_a, phase_deg);
}

sdd_status sdd_solve_multi_freq(sdd_ctx_t ctx, const sdd_request *req, uint32_t n_freq, const double *freqs,
                                const double *const *g_tables, sdd_result *res) {
  if (!ctx || !req) return fail(SDD_E_INVALID, "NULL argument");
  if (n_freq && (!freqs || !g_tables || !res)) return fail(SDD_E_INVALID, "NULL frequencies, tables or results");
  if (req->target_rel_se > 0.0) return fail(SDD_E_INVALID, "multi-frequency solves take fixed-path requests");
  const double ref = req->alpha_direct > 0.0 ? req->alpha_direct : req->freq_hz;
  if (!(ref > 0.0) || !std::isfinite(ref))
    return fail(SDD_E_INVALID, "multi-frequency solves need a positive request frequency (or alpha)");
  for (uint32_t k = 0; k < n_freq; ++k) {
    if (!(freqs[k] > 0.0) || !std::isfinite(freqs[k])) return fail(SDD_E_INVALID, "frequency %u is not positive", k);
    if (!g_tables[k]) return fail(SDD_E_INVALID, "g_tables[%u] is NULL", k);
    for (uint64_t i = 0; i < 8ull * req->g_samples; ++i)
      if (!std::isfinite(g_tables[k][i])) return fail(SDD_E_INVALID, "g_tables[%u] holds a non-finite value", k);
    if (!res[k].mean && req->n_nodes) return fail(SDD_E_INVALID, "result %u: mean is NULL", k);
    if (res[k].path_records) return fail(SDD_E_INVALID, "result %u: no path records in multi-frequency solves", k);
  }
  std::unique_ptr<Prepared> P;
  sdd_status st = prepare(ctx, req, P);
  if (st != SDD_OK) return st;
  P->dreq.fanout = 1u;
  ExecGuard ex(ctx);
  HIP_TRY(hipSetDevice(ctx->device));
  st = upload_pass(ctx, *P);
  std::vector<Prepared *> Ps{P.get()};
  if (st == SDD_OK) st = run_persistent(ctx, Ps);
  const uint32_t n = (uint32_t)P->pbeg.size();
  const uint64_t n_jobs = (uint64_t)n * n_freq;
  const size_t tab = (size_t)8 * req->g_samples;
  char *d_g = nullptr, *d_jobs = nullptr, *d_out = nullptr;
  std::vector<NodeOut> rows(n_jobs);
  if (st == SDD_OK && n_jobs) {
    d_g = ctx->alloc(n_freq * tab * sizeof(double));
    d_jobs = ctx->alloc(n_jobs * sizeof(FanJob));
    d_out = ctx->alloc(n_jobs * sizeof(NodeOut));
    if (!d_g || !d_jobs || !d_out) st = fail(SDD_E_NOMEM, "no workspace left for the multi-frequency reduction");
  }
  if (st == SDD_OK && n_jobs) {
    std::vector<FanJob> jobs(n_jobs);
    for (uint32_t k = 0; k < n_freq; ++k)
      for (uint32_t j = 0; j < n; ++j) {
        FanJob &J = jobs[(uint64_t)k * n + j];
        J.recs = reinterpret_cast<const PathRec *>(P->d_recs) + P->rec_off[j];
        J.count = P->pcnt[j];
        J.g = reinterpret_cast<const double *>(d_g) + k * tab;
        J.scale = freqs[k] / ref;
        J.out = reinterpret_cast<NodeOut *>(d_out) + (uint64_t)k * n + j;
      }
    hipError_t e = hipSuccess;
    for (uint32_t k = 0; k < n_freq && e == hipSuccess; ++k)
      e = hipMemcpyAsync(d_g + k * tab * sizeof(double), g_tables[k], tab * sizeof(double), hipMemcpyHostToDevice,
                         ctx->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_jobs, jobs.data(), n_jobs * sizeof(FanJob), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipEventRecord(ctx->ev[2], ctx->stream);
    if (e == hipSuccess)
      e = launch_reduce_fanout(reinterpret_cast<const FanJob *>(d_jobs), (uint32_t)n_jobs, (int)P->dreq.M,
                               P->dreq.y_lo, P->dreq.y_hi, P->dreq.z_lo, P->dreq.z_hi, ctx->stream);
    if (e == hipSuccess) e = hipEventRecord(ctx->ev[3], ctx->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(rows.data(), d_out, n_jobs * sizeof(NodeOut), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) st = fail(SDD_E_DEVICE, "multi-frequency reduction: %s", hipGetErrorString(e));
    float ms = 0.f;
    if (st == SDD_OK && hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]) == hipSuccess) ctx->stats.last_reduce_ms = ms;
    if (st == SDD_OK && n) {
      uint64_t steps = 0;
      for (uint32_t j = 0; j < n; ++j) steps += rows[j].steps;
      ctx->stats.last_walk_steps = steps;
    }
  }
  ctx->release(d_g);
  ctx->release(d_jobs);
  ctx->release(d_out);
  if (st == SDD_OK)
    for (uint32_t k = 0; k < n_freq; ++k) {
      const NodeOut *rk = rows.data() + (uint64_t)k * n;
      scatter_rows(n, rk, &res[k]);
      // the phase per step scales with the frequency; each frequency has its tables
      double rho = 0.0;
      for (uint32_t r = 0; r <= P->dreq.nprims; ++r) rho = std::max(rho, P->dreq.c[r]);
      fill_diag(res[k].diag, rho * (freqs[k] / ref), g_norm(std::vector<double>(g_tables[k], g_tables[k] + tab)),
                n, rk);
    }
  release_all(ctx, *P);
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
  ExecGuard ex(ctx);
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
    ++ctx->epoch;
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
  for (auto *dq : {&ctx->queue, &ctx->requeue}) {
    auto q = std::find(dq->begin(), dq->end(), T);
    if (q == dq->end()) continue;
    // not admitted (or given back for re-admission): finish it now; the
    // requests behind it may fit now
    dq->erase(q);
    finish_ticket(ctx, *T, SDD_E_CANCELLED, nullptr);
    T->P.reset();
    ++ctx->epoch;
    ctx->done_cv.notify_all();
    ctx->cv.notify_all();
    break;
  }
  return SDD_OK;
}

// ---------------------------------------------------------------------------
// Discontinuous kappa: one vertical interface, FP64 walk (sdd_kappa.hip).
// ---------------------------------------------------------------------------
static sdd_status validate_kappa(const sdd_kappa_request *r) {
  auto fin = [](double v) { return std::isfinite(v); };
  if (!(fin(r->y_lo) && fin(r->y_hi) && fin(r->z_lo) && fin(r->z_hi) && r->y_lo < r->y_hi && r->z_lo < r->z_hi))
    return fail(SDD_E_INVALID, "Omega must be a finite rectangle");
  if (!(fin(r->y_if) && r->y_lo < r->y_if && r->y_if < r->y_hi))
    return fail(SDD_E_INVALID, "the interface must lie strictly inside Omega");
  for (int i = 0; i < 2; ++i) {
    if (!(fin(r->kappa[i]) && r->kappa[i] > 0.0)) return fail(SDD_E_INVALID, "kappa must be finite and > 0");
    if (!(fin(r->lambda_re[i]) && r->lambda_re[i] >= 0.0) || !fin(r->lambda_im[i]))
      return fail(SDD_E_INVALID, "lambda must be finite with a real part >= 0");
  }
  if (!(fin(r->dt) && r->dt > 0.0)) return fail(SDD_E_INVALID, "dt must be finite and > 0");
  const double half = 0.5 * std::min(r->y_hi - r->y_lo, r->z_hi - r->z_lo);
  if (!(7.0 * std::sqrt(std::max(r->kappa[0], r->kappa[1]) * r->dt) < half))
    return fail(SDD_E_INVALID, "dt too large: 7 sqrt(kappa dt) must be below half the shorter side");
  if (r->stream >= (1u << 30)) return fail(SDD_E_INVALID, "stream must be < 2^30");
  if (r->precision != SDD_FP64 && r->precision != SDD_FP32_MIXED)
    return fail(SDD_E_INVALID, "precision must be SDD_FP64 or SDD_FP32_MIXED");
  if (r->g_samples < 2 || !r->g_tables) return fail(SDD_E_INVALID, "g_tables need >= 2 samples per wall");
  for (size_t k = 0; k < (size_t)8 * r->g_samples; ++k)
    if (!fin(r->g_tables[k])) return fail(SDD_E_INVALID, "g_tables must be finite");
  if (r->n_nodes && !r->nodes_yz) return fail(SDD_E_INVALID, "nodes_yz is NULL");
  uint64_t total = 0;
  for (uint32_t j = 0; j < r->n_nodes; ++j) {
    const double y = r->nodes_yz[2 * j], z = r->nodes_yz[2 * j + 1];
    if (!(y > r->y_lo && y < r->y_hi && z > r->z_lo && z < r->z_hi))
      return fail(SDD_E_INVALID, "node %u is not strictly inside Omega", j);
    const uint32_t b = r->path_begin ? r->path_begin[j] : 0u;
    const uint32_t c = r->path_count ? r->path_count[j] : r->paths_uniform;
    if (c == 0) return fail(SDD_E_INVALID, "node %u has no paths", j);
    if ((uint64_t)b + c > (1ull << 32)) return fail(SDD_E_INVALID, "node %u: path range passes 2^32", j);
    total += c;
  }
  if (total > (1ull << 40)) return fail(SDD_E_INVALID, "more than 2^40 paths");
  return SDD_OK;
}

sdd_status sdd_solve_kappa(sdd_ctx_t ctx, const sdd_kappa_request *r, sdd_result *res) {
  if (!ctx || !r || !res) return fail(SDD_E_INVALID, "NULL argument");
  sdd_status st = validate_kappa(r);
  if (st != SDD_OK) return st;
  const uint32_t n = r->n_nodes;
  if (n == 0) return SDD_OK;
  if (!res->mean) return fail(SDD_E_INVALID, "result mean is NULL");

  // tiles of one node's paths, record slots node-major in path order; claimed
  // longest expected paths first, sizes guided as for sdd_solve
  const uint32_t tile_paths = ctx->tuning.tile_paths ? ctx->tuning.tile_paths : 512u;
  std::vector<DevTile> tiles;
  std::vector<uint64_t> rec_off(n + 1, 0);
  uint64_t total = 0;
  for (uint32_t j = 0; j < n; ++j) {
    rec_off[j] = total;
    total += r->path_count ? r->path_count[j] : r->paths_uniform;
  }
  rec_off[n] = total;
  {
    DevReq walls{};
    walls.y_lo = r->y_lo; walls.y_hi = r->y_hi; walls.z_lo = r->z_lo; walls.z_hi = r->z_hi;
    std::vector<uint32_t> order(n);
    std::vector<double> key(n);
    for (uint32_t j = 0; j < n; ++j) {
      const double y = r->nodes_yz[2 * j], z = r->nodes_yz[2 * j + 1];
      order[j] = j;
      key[j] = exit_time_estimate(walls, y, z) / r->kappa[y < r->y_if ? 0 : 1];
    }
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return key[a] > key[b]; });
    const uint64_t waves = launch_waves_estimate(ctx);
    uint64_t remaining = total;
    for (uint32_t j : order) {
      const uint32_t b = r->path_begin ? r->path_begin[j] : 0u;
      const uint32_t c = r->path_count ? r->path_count[j] : r->paths_uniform;
      uint32_t k = 0;
      while (k < c) {
        const uint32_t cnt = std::min(guided_tile(remaining, waves, tile_paths), c - k);
        DevTile t{};
        t.node = j;
        t.p0 = b + k;
        t.count = cnt;
        t.rec0 = rec_off[j] + k;
        tiles.push_back(t);
        k += cnt;
        remaining -= cnt;
      }
    }
  }
  if (tiles.size() >= (1ull << 32)) return fail(SDD_E_INVALID, "too many tiles");

  KReq K{};
  K.y_lo = r->y_lo; K.y_hi = r->y_hi; K.z_lo = r->z_lo; K.z_hi = r->z_hi; K.y_if = r->y_if;
  K.dt = r->dt;
  for (int i = 0; i < 2; ++i) {
    K.kdt[i] = r->kappa[i] * r->dt;
    K.s[i] = std::sqrt(K.kdt[i]);
    // -log u <= 22.87 for every uniform ((w + 1/2) 2^-32), so a bridge can
    // only hit when 2 d0 d1 <= 22.87 kappa dt
    K.thr[i] = 22.9 * K.kdt[i];
    K.p[i] = r->kappa[i] / (r->kappa[0] + r->kappa[1]);
    K.kappa[i] = r->kappa[i];
    K.lre[i] = r->lambda_re[i];
    K.lim[i] = r->lambda_im[i];
  }
  K.M = r->g_samples - 1u;
  K.n_tiles = (uint32_t)tiles.size();
  K.key0 = (uint32_t)(r->seed & 0xFFFFFFFFull);
  K.key1 = (uint32_t)(r->seed >> 32);
  K.ctr3 = 4u * r->stream;
  K.max_steps = r->max_steps ? r->max_steps : kDefaultMaxSteps;
  K.equal_kappa = r->kappa[0] == r->kappa[1] ? 1u : 0u;
  K.ymid = 0.5 * (r->y_lo + r->y_hi);
  K.zmid = 0.5 * (r->z_lo + r->z_hi);
  K.fhy = (float)(0.5 * (r->y_hi - r->y_lo));
  K.fhz = (float)(0.5 * (r->z_hi - r->z_lo));
  K.fa_if = (float)(r->y_if - K.ymid);
  K.fdt = (float)r->dt;
  K.frdt = (float)(1.0 / r->dt);
  for (int i = 0; i < 2; ++i) {
    K.fK[i] = (float)(K.s[i] * std::sqrt(2.0 * std::log(2.0)));
    K.fs[i] = (float)K.s[i];
    // FP32 uniforms are at least 2^-24, so -ln U <= 16.64: no bridge hit is
    // possible once 2 d0 d1 > 16.7 kappa_i dt
    K.fthr[i] = (float)(16.7 * K.kdt[i]);
    K.fkdt[i] = (float)K.kdt[i];
    K.fkappa[i] = (float)r->kappa[i];
    K.fp[i] = (float)K.p[i];
  }

  ExecGuard ex(ctx);
  HIP_TRY(hipSetDevice(ctx->device));
  const size_t g_bytes = (size_t)8 * r->g_samples * sizeof(double);
  char *d_g = ctx->alloc(g_bytes);
  char *d_nodes = ctx->alloc((size_t)2 * n * sizeof(double));
  char *d_tiles = ctx->alloc(tiles.size() * sizeof(DevTile));
  char *d_recs = ctx->alloc(total * sizeof(PathRec));
  char *d_req = ctx->alloc(sizeof(KReq) + sizeof(uint32_t) * 64);
  char *d_out = ctx->alloc((size_t)n * sizeof(NodeOut));
  char *d_jobs = ctx->alloc((size_t)n * sizeof(NodeJob));
  auto release = [&]() {
    for (char *p : {d_g, d_nodes, d_tiles, d_recs, d_req, d_out, d_jobs}) ctx->release(p);
  };
  if (!d_g || !d_nodes || !d_tiles || !d_recs || !d_req || !d_out || !d_jobs) {
    release();
    return fail(SDD_E_NOMEM, "workspace too small for %llu paths", (unsigned long long)total);
  }
  uint32_t *d_ctr = reinterpret_cast<uint32_t *>(d_req + sizeof(KReq));   // the tile counter
  K.g = reinterpret_cast<const double *>(d_g);
  K.nodes = reinterpret_cast<const double *>(d_nodes);
  K.tiles = reinterpret_cast<const DevTile *>(d_tiles);
  K.recs = reinterpret_cast<PathRec *>(d_recs);
  K.tile_counter = d_ctr;

  std::vector<NodeJob> jobs(n);
  for (uint32_t j = 0; j < n; ++j) {
    jobs[j] = NodeJob{};
    jobs[j].recs0 = reinterpret_cast<const PathRec *>(d_recs) + rec_off[j];
    jobs[j].count0 = rec_off[j + 1] - rec_off[j];
    jobs[j].out = reinterpret_cast<NodeOut *>(d_out) + j;
  }
  const uint32_t threads = kappa_threads();
  const uint32_t waves_per_block = threads / 64u;
  const int bpc = std::max(kappa_blocks_per_cu((int)r->precision), 1);
  uint32_t blocks = (uint32_t)std::max(ctx->cus, 1) * (uint32_t)bpc;
  blocks = std::max<uint32_t>(1u, std::min<uint32_t>(blocks, (K.n_tiles + waves_per_block - 1) / waves_per_block));
  const uint32_t zero = 0u;
  std::vector<NodeOut> rows(n);
  hipStream_t s = ctx->stream;
  hipError_t e = hipMemcpyAsync(d_g, r->g_tables, g_bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_nodes, r->nodes_yz, (size_t)2 * n * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_tiles, tiles.data(), tiles.size() * sizeof(DevTile), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_req, &K, sizeof(KReq), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_ctr, &zero, sizeof(zero), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_jobs, jobs.data(), jobs.size() * sizeof(NodeJob), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(ctx->ev[0], s);
  if (e == hipSuccess) e = launch_walk_kappa((int)r->precision, reinterpret_cast<const KReq *>(d_req), blocks, s);
  if (e == hipSuccess) e = hipEventRecord(ctx->ev[1], s);
  if (e == hipSuccess) e = launch_reduce(reinterpret_cast<const NodeJob *>(d_jobs), n, s);
  if (e == hipSuccess) e = hipEventRecord(ctx->ev[2], s);
  if (e == hipSuccess) e = hipMemcpyAsync(rows.data(), d_out, (size_t)n * sizeof(NodeOut), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && res->path_records)
    e = hipMemcpyAsync(res->path_records, d_recs, total * sizeof(PathRec), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    release();
    return fail(SDD_E_DEVICE, "kappa walk: %s", hipGetErrorString(e));
  }
  float ms = 0.f, rms = 0.f;
  if (hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]) == hipSuccess) ctx->stats.last_walk_ms = ms;
  if (hipEventElapsedTime(&rms, ctx->ev[1], ctx->ev[2]) == hipSuccess) ctx->stats.last_reduce_ms = rms;
  uint64_t steps = 0;
  for (const NodeOut &o : rows) steps += o.steps;
  ctx->stats.last_walk_steps = steps;
  ctx->stats.last_walk_paths = total;
  ctx->stats.last_blocks = blocks;
  ctx->stats.last_threads = threads;
  ctx->stats.launches += 1;
  scatter_rows(n, rows.data(), res);
  {
    double gn = 0.0;
    for (size_t k = 0; k + 1 < (size_t)8 * r->g_samples; k += 2)
      gn = std::max(gn, std::hypot(r->g_tables[k], r->g_tables[k + 1]));
    const double rho = std::max(std::hypot(r->lambda_re[0], r->lambda_im[0]),
                                std::hypot(r->lambda_re[1], r->lambda_im[1])) * r->dt;
    fill_diag(res->diag, rho, gn, n, rows.data());
  }
  release();
  return SDD_OK;
}

// sdd_solve with every device buffer in the static scratch of this device
// instead of the context's workspace; the same kernels in the same launch
// sequence, so the results are bitwise those of sdd_solve.
sdd_status sdd_solve_noalloc(sdd_ctx_t ctx, const sdd_request *req, sdd_result *res) {
  if (!ctx || !req || !res) return fail(SDD_E_INVALID, "NULL argument");
  if (req->target_rel_se > 0.0) return fail(SDD_E_INVALID, "sdd_solve_noalloc takes fixed path counts");
  if (!res->mean && req->n_nodes) return fail(SDD_E_INVALID, "result mean is NULL");
  std::unique_ptr<Prepared> P;
  sdd_status st = prepare(ctx, req, P);
  if (st != SDD_OK) return st;
  if (!ctx->scratch) return fail(SDD_E_DEVICE, "no static scratch on device %d", ctx->device);
  const uint32_t n = req->n_nodes;
  build_tiles(*P, tile_size(ctx, *P), launch_waves_estimate(ctx));
  // layout of the scratch, 256-byte aligned pieces
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += Arena::round(b ? b : 1);
    return o;
  };
  const size_t o_req = take(sizeof(DevReq)), o_ctr = take(sizeof(uint32_t)),
               o_done = take(sizeof(unsigned long long)), o_ws = take(2 * sizeof(uint32_t)),
               o_g = take(P->g.size() * sizeof(double)), o_nodes = take(P->nodes.size() * sizeof(double)),
               o_grid = take(P->grid.size() * sizeof(SigmaCell)), o_ext = take(P->grid_ext.size() * sizeof(SigmaCell)),
               o_tiles = take(P->tiles.size() * sizeof(DevTile)),
               o_recs = take(P->n_paths * sizeof(PathRec)), o_jobs = take((size_t)n * sizeof(NodeJob)),
               o_out = take((size_t)n * sizeof(NodeOut));
  if (off > scratch_bytes())
    return fail(SDD_E_NOMEM, "request needs %zu bytes of static scratch; sdd_solve_noalloc has %zu", off,
                scratch_bytes());
  if (n == 0) {
    scatter(*P, nullptr, res);
    return SDD_OK;
  }
  ExecGuard ex(ctx);
  HIP_TRY(hipSetDevice(ctx->device));
  std::lock_guard<std::mutex> use(scratch_lock(ctx->device));
  char *base = ctx->scratch;
  DevReq q = P->dreq;
  q.g = reinterpret_cast<const double *>(base + o_g);
  q.nodes = reinterpret_cast<const double *>(base + o_nodes);
  q.tiles = reinterpret_cast<const DevTile *>(base + o_tiles);
  q.recs = reinterpret_cast<PathRec *>(base + o_recs);
  q.grid = P->grid.empty() ? nullptr : reinterpret_cast<const SigmaCell *>(base + o_grid);
  q.grid_ext = P->grid_ext.empty() ? nullptr : reinterpret_cast<const SigmaCell *>(base + o_ext);
  q.n_tiles = (uint32_t)P->tiles.size();
  q.tile_counter = reinterpret_cast<uint32_t *>(base + o_ctr);
  q.done_counter = reinterpret_cast<unsigned long long *>(base + o_done);
  uint32_t blocks, threads;
  launch_shape(ctx, (int)q.precision, q.sig, 0, blocks, threads);
  const uint32_t ws[2] = {0u, blocks * (threads / 64)};
  std::vector<NodeJob> jobs(n);
  for (uint32_t j = 0; j < n; ++j) {
    jobs[j] = NodeJob{};
    jobs[j].recs0 = reinterpret_cast<const PathRec *>(base + o_recs) + P->rec_off[j];
    jobs[j].count0 = P->pcnt[j];
    jobs[j].out = reinterpret_cast<NodeOut *>(base + o_out) + j;
  }
  std::vector<NodeOut> rows(n);
  unsigned long long done = 0;
  hipStream_t s = ctx->stream;
  hipError_t e = hipMemcpyAsync(base + o_g, P->g.data(), P->g.size() * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + o_nodes, P->nodes.data(), P->nodes.size() * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !P->grid.empty())
    e = hipMemcpyAsync(base + o_grid, P->grid.data(), P->grid.size() * sizeof(SigmaCell), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !P->grid_ext.empty())
    e = hipMemcpyAsync(base + o_ext, P->grid_ext.data(), P->grid_ext.size() * sizeof(SigmaCell),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !P->tiles.empty())
    e = hipMemcpyAsync(base + o_tiles, P->tiles.data(), P->tiles.size() * sizeof(DevTile), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(base + o_req, &q, sizeof(DevReq), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(base + o_ws, ws, sizeof(ws), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(base + o_jobs, jobs.data(), n * sizeof(NodeJob), hipMemcpyHostToDevice, s);
  // the counters keep the previous call's values: a fill kernel zeroes them
  if (e == hipSuccess)
    e = launch_reset(reinterpret_cast<uint32_t *>(base + o_ctr), reinterpret_cast<unsigned long long *>(base + o_done),
                     1u, s);
  if (e == hipSuccess) e = hipEventRecord(ctx->ev[0], s);
  if (e == hipSuccess)
    e = launch_walk_persist((int)q.precision, q.sig, reinterpret_cast<const DevReq *>(base + o_req), 1u,
                            reinterpret_cast<const uint32_t *>(base + o_ws), 0u, refill_mask(ctx), blocks, threads, 0u,
                            s);
  if (e == hipSuccess) e = hipEventRecord(ctx->ev[1], s);
  if (e == hipSuccess) e = launch_reduce(reinterpret_cast<const NodeJob *>(base + o_jobs), n, s);
  if (e == hipSuccess) e = hipEventRecord(ctx->ev[2], s);
  if (e == hipSuccess) e = hipMemcpyAsync(rows.data(), base + o_out, n * sizeof(NodeOut), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&done, base + o_done, sizeof(done), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && res->path_records && P->n_paths)
    e = hipMemcpyAsync(res->path_records, base + o_recs, P->n_paths * sizeof(PathRec), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    // work queued before the failing call may still use the scratch: let it
    // drain before the lock is released
    (void)hipStreamSynchronize(s);
    return fail(SDD_E_DEVICE, "sdd_solve_noalloc: %s", hipGetErrorString(e));
  }
  if (done != P->n_paths)
    return fail(SDD_E_DEVICE, "%llu of %llu paths completed", done, (unsigned long long)P->n_paths);
  float ms = 0.f, rms = 0.f;
  if (hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]) == hipSuccess) ctx->stats.last_walk_ms = ms;
  if (hipEventElapsedTime(&rms, ctx->ev[1], ctx->ev[2]) == hipSuccess) ctx->stats.last_reduce_ms = rms;
  uint64_t steps = 0;
  for (const NodeOut &o : rows) steps += o.steps;
  ctx->stats.last_walk_steps = steps;
  ctx->stats.last_walk_paths = P->n_paths;
  ctx->stats.last_blocks = blocks;
  ctx->stats.last_threads = threads;
  ctx->stats.launches += 1;
  scatter(*P, rows.data(), res);
  return SDD_OK;
}

sdd_status sdd_request_footprint(sdd_ctx_t ctx, const sdd_request *req, uint64_t *bytes) {
  if (!ctx || !req || !bytes) return fail(SDD_E_INVALID, "NULL argument");
  std::unique_ptr<Prepared> P;
  sdd_status st = prepare(ctx, req, P);
  if (st != SDD_OK) return st;
  *bytes = footprint(ctx, *P, true);
  return SDD_OK;
}

sdd_status sdd_set_tuning(sdd_ctx_t ctx, const sdd_tuning *t) {
  if (!ctx || !t) return fail(SDD_E_INVALID, "NULL argument");
  if (t->block_threads && (t->block_threads % 64 || t->block_threads > 256))
    return fail(SDD_E_INVALID, "block_threads must be a multiple of 64, at most 256 (the walker's launch bound)");
  if (t->blocks_per_cu > 64) return fail(SDD_E_INVALID, "blocks_per_cu at most 64");
  if (t->tile_paths > (1u << 24)) return fail(SDD_E_INVALID, "tile_paths at most 2^24");
  if (t->refill_every > 64 || (t->refill_every & (t->refill_every - 1)) != 0)
    return fail(SDD_E_INVALID, "refill_every must be a power of 2, at most 64");
  ExecGuard ex(ctx);
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->tuning = *t;
  if (!ctx->tuning.block_threads) ctx->tuning.block_threads = 256;
  if (!ctx->tuning.tile_paths) ctx->tuning.tile_paths = 512;
  if (!ctx->tuning.slice_iters) ctx->tuning.slice_iters = 4096;
  if (!ctx->tuning.refill_every) ctx->tuning.refill_every = 1;
  return SDD_OK;
}

sdd_status sdd_get_stats(sdd_ctx_t ctx, sdd_stats *out) {
  if (!ctx || !out) return fail(SDD_E_INVALID, "NULL argument");
  ExecGuard ex(ctx);
  *out = ctx->stats;
  std::lock_guard<std::mutex> lk(ctx->mu);
  out->served_in_flight_max = ctx->served_in_flight_max;
  out->served_waits = ctx->served_waits;
  out->served_requeues = ctx->served_requeues;
  out->served_walk_ms = ctx->served_walk_ms;
  out->served_slices = ctx->served_slices;
  return SDD_OK;
}

sdd_status sdd_get_tuning(sdd_ctx_t ctx, sdd_tuning *t) {
  if (!ctx || !t) return fail(SDD_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(ctx->mu);
  *t = ctx->tuning;
  return SDD_OK;
}

sdd_status sdd_autotune(sdd_ctx_t ctx, const sdd_request *req, uint32_t sample_paths, sdd_tuning *chosen,
                        sdd_tune_trial *trials, uint32_t max_trials, uint32_t *n_trials) {
  if (!ctx || !req) return fail(SDD_E_INVALID, "NULL argument");
  if (req->n_nodes == 0) return fail(SDD_E_INVALID, "autotune needs a request with nodes");
  if (trials == nullptr && max_trials) return fail(SDD_E_INVALID, "trials is NULL");
  if (n_trials) *n_trials = 0;
  sdd_request s = *req;
  s.target_rel_se = 0.0;
  if (!sample_paths) {
    uint32_t b, t;
    launch_shape(ctx, (int)req->precision, -1, 0, b, t);
    sample_paths = (uint32_t)std::min<uint64_t>(1u << 24, (4ull * b * t + req->n_nodes - 1) / req->n_nodes);
  }
  std::vector<uint32_t> cnt(req->n_nodes);
  uint64_t total = 0;
  for (uint32_t j = 0; j < req->n_nodes; ++j) {
    const uint32_t c = req->path_count ? req->path_count[j] : req->paths_uniform;
    cnt[j] = std::min(c, sample_paths);
    total += cnt[j];
  }
  if (total == 0) return fail(SDD_E_INVALID, "autotune needs a request with paths");
  s.path_count = cnt.data();
  std::unique_ptr<Prepared> P;
  sdd_status st = prepare(ctx, &s, P);
  if (st != SDD_OK) return st;

  ExecGuard ex(ctx);
  HIP_TRY(hipSetDevice(ctx->device));
  const sdd_tuning base = ctx->tuning;
  uint32_t n_done = 0;
  auto trial = [&](const sdd_tuning &t, double &ms) -> sdd_status {
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->tuning = t;
    }
    std::vector<Prepared *> Ps{P.get()};
    std::vector<std::vector<NodeOut>> rows;
    sdd_status r = execute(ctx, Ps, rows);
    release_all(ctx, *P);
    if (r != SDD_OK) return r;
    ms = ctx->stats.last_walk_ms;
    if (n_done < max_trials) {
      trials[n_done].tuning = t;
      trials[n_done].walk_ms = ms;
      trials[n_done].walk_steps_per_s = ms > 0 ? (double)ctx->stats.last_walk_steps / (ms * 1e-3) : 0.0;
    }
    ++n_done;
    return SDD_OK;
  };
  // Coordinate descent from the current tuning: launch block size, then
  // tile size, then refill cadence, each swept with the others held.
  sdd_tuning best = base;
  double best_ms = 0.0;
  double warm = 0.0;
  st = trial(best, warm);   // warm-up (first-touch of the workspace, clocks)
  if (st == SDD_OK) st = trial(best, best_ms);
  const uint32_t threads_c[] = {256, 128, 64};
  const uint32_t tiles_c[] = {128, 512, 2048, 8192};
  const uint32_t refill_c[] = {1, 2, 4, 8};
  for (int axis = 0; axis < 3 && st == SDD_OK; ++axis) {
    const uint32_t *vals = axis == 0 ? threads_c : axis == 1 ? tiles_c : refill_c;
    const int nv = axis == 0 ? 3 : 4;
    sdd_tuning round_best = best;
    for (int k = 0; k < nv && st == SDD_OK; ++k) {
      sdd_tuning t = best;
      uint32_t &field = axis == 0 ? t.block_threads : axis == 1 ? t.tile_paths : t.refill_every;
      if (field == vals[k]) continue;
      field = vals[k];
      if (axis == 0) t.blocks_per_cu = 0;   // occupancy of the new block size
      double ms = 0.0;
      st = trial(t, ms);
      if (st == SDD_OK && ms < best_ms) { best_ms = ms; round_best = t; }
    }
    best = round_best;
  }
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->tuning = st == SDD_OK ? best : base;
  }
  if (n_trials) *n_trials = std::min(n_done, max_trials);
  if (st != SDD_OK) return st;
  if (chosen) *chosen = best;
  return SDD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Prepared batches replayed as HIP graphs.
// ---------------------------------------------------------------------------
struct sdd_batch {
  sdd_ctx *ctx = nullptr;
  std::vector<std::unique_ptr<Prepared>> Ps;
  struct Group {
    int prec;
    int sig = -1;
    uint32_t lds_bytes = 0;
    std::vector<Prepared *> P;
    char *d_reqs = nullptr, *d_ctr = nullptr, *d_done = nullptr, *d_ws = nullptr;
    uint32_t blocks = 0, threads = 0;
  };
  std::vector<Group> groups;
  char *d_jobs = nullptr, *d_out = nullptr, *d_done_all = nullptr;
  NodeOut *h_out = nullptr;                // pinned
  unsigned long long *h_done = nullptr;    // pinned, one per request (group order)
  uint64_t total_nodes = 0;
  hipStream_t cap = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};   // around each replay, on the context's stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t held = 0;                       // workspace counted as held for the batch's life
};

static void batch_free(sdd_batch *b) {
  if (!b) return;
  sdd_ctx *ctx = b->ctx;
  if (b->held) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->held_long -= std::min(ctx->held_long, b->held);
  }
  // teardown: nothing to do on failure
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (auto &e : b->ev)
    if (e) (void)hipEventDestroy(e);
  if (b->h_out) (void)hipHostFree(b->h_out);
  if (b->h_done) (void)hipHostFree(b->h_done);
  for (auto &g : b->groups) {
    ctx->release(g.d_reqs);
    ctx->release(g.d_ctr);
    ctx->release(g.d_ws);
  }
  ctx->release(b->d_done_all);
  ctx->release(b->d_jobs);
  ctx->release(b->d_out);
  for (auto &P : b->Ps) release_all(ctx, *P);
  delete b;
}

extern "C" {

sdd_status sdd_batch_create(sdd_ctx_t ctx, uint32_t n, const sdd_request *reqs, sdd_batch_t *out) {
  if (!ctx || !out || (n && !reqs)) return fail(SDD_E_INVALID, "NULL argument");
  *out = nullptr;
  auto *b = new sdd_batch();
  b->ctx = ctx;
  b->Ps.resize(n);
  for (uint32_t i = 0; i < n; ++i) {
    if (reqs[i].target_rel_se > 0.0) {
      batch_free(b);
      return fail(SDD_E_INVALID, "request %u: a prepared batch takes fixed path counts", i);
    }
    sdd_status st = prepare(ctx, &reqs[i], b->Ps[i]);
    if (st != SDD_OK) { batch_free(b); return st; }
  }
  ExecGuard ex(ctx);
  auto bail = [&](sdd_status st) { batch_free(b); return st; };
  if (hipSetDevice(ctx->device) != hipSuccess) return bail(fail(SDD_E_DEVICE, "hipSetDevice failed"));
  for (auto &P : b->Ps) {
    sdd_status st = upload_pass(ctx, *P);
    if (st != SDD_OK) return bail(st);
    b->total_nodes += P->pbeg.size();
  }
  // per-precision descriptors, counters and wave shares
  b->d_done_all = ctx->alloc(std::max<size_t>(n, 1) * sizeof(unsigned long long));
  if (!b->d_done_all) return bail(fail(SDD_E_NOMEM, "no workspace for the batch counters"));
  uint32_t done_slot = 0;
  std::vector<uint32_t> done_index(n, 0);
  for (int prec : {SDD_FP32_MIXED, SDD_FP64}) {
    sdd_batch::Group g;
    g.prec = prec;
    for (uint32_t i = 0; i < n; ++i)
      if ((int)b->Ps[i]->dreq.precision == prec) g.P.push_back(b->Ps[i].get());
    if (g.P.empty()) continue;
    const uint32_t m = (uint32_t)g.P.size();
    g.sig = launch_sig(g.P.begin(), g.P.end(), [](const Prepared *P) { return P; }, g.lds_bytes);
    launch_shape(ctx, prec, g.sig, g.lds_bytes, g.blocks, g.threads);
    const uint32_t waves = g.blocks * (g.threads / 64);
    g.d_reqs = ctx->alloc(m * sizeof(DevReq));
    g.d_ctr = ctx->alloc(m * sizeof(uint32_t));
    g.d_ws = ctx->alloc((m + 1) * sizeof(uint32_t));
    g.d_done = b->d_done_all + (size_t)done_slot * sizeof(unsigned long long);
    if (!g.d_reqs || !g.d_ctr || !g.d_ws) {
      b->groups.push_back(g);
      return bail(fail(SDD_E_NOMEM, "no workspace for the batch descriptors"));
    }
    std::vector<DevReq> dq(m);
    std::vector<uint32_t> ws(m + 1, 0);
    double total = 0.0, acc = 0.0;
    for (auto *P : g.P) total += (double)P->n_paths;
    for (uint32_t i = 0; i < m; ++i) {
      dq[i] = g.P[i]->dreq;
      if (g.sig == kSigGenericLds) dq[i].sig = kSigGenericLds;
      dq[i].tile_counter = reinterpret_cast<uint32_t *>(g.d_ctr) + i;
      dq[i].done_counter = reinterpret_cast<unsigned long long *>(g.d_done) + i;
      ws[i] = total > 0 ? (uint32_t)std::llround(acc / total * waves) : 0u;
      acc += (double)g.P[i]->n_paths;
      for (uint32_t k = 0; k < n; ++k)
        if (b->Ps[k].get() == g.P[i]) done_index[k] = done_slot + i;
    }
    ws[m] = waves;
    done_slot += m;
    if (hipMemcpy(g.d_reqs, dq.data(), m * sizeof(DevReq), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g.d_ws, ws.data(), (m + 1) * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess) {
      b->groups.push_back(g);
      return bail(fail(SDD_E_DEVICE, "batch descriptor upload failed"));
    }
    b->groups.push_back(g);
  }
  // reduction jobs in request order
  b->d_out = ctx->alloc(std::max<uint64_t>(b->total_nodes, 1) * sizeof(NodeOut));
  b->d_jobs = ctx->alloc(std::max<uint64_t>(b->total_nodes, 1) * sizeof(NodeJob));
  if (!b->d_out || !b->d_jobs) return bail(fail(SDD_E_NOMEM, "no workspace for the batch reduction"));
  std::vector<NodeJob> jobs;
  uint64_t row = 0;
  for (auto &P : b->Ps)
    for (uint32_t j = 0; j < P->pbeg.size(); ++j, ++row) {
      NodeJob J{};
      J.out = reinterpret_cast<NodeOut *>(b->d_out) + row;
      J.recs0 = reinterpret_cast<const PathRec *>(P->d_recs) + P->rec_off[j];
      J.count0 = P->pcnt[j];
      jobs.push_back(J);
    }
  if (!jobs.empty() &&
      hipMemcpy(b->d_jobs, jobs.data(), jobs.size() * sizeof(NodeJob), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(SDD_E_DEVICE, "batch job upload failed"));
  if (hipHostMalloc(reinterpret_cast<void **>(&b->h_out), std::max<uint64_t>(b->total_nodes, 1) * sizeof(NodeOut),
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void **>(&b->h_done), std::max<size_t>(n, 1) * sizeof(unsigned long long),
                    hipHostMallocDefault) != hipSuccess)
    return bail(fail(SDD_E_DEVICE, "pinned host buffers"));
  // capture: counter reset (a kernel, not a memset), walks, reduction, copies
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(SDD_E_DEVICE, "capture stream"));
  if (hipEventCreate(&b->ev[0]) != hipSuccess || hipEventCreate(&b->ev[1]) != hipSuccess)
    return bail(fail(SDD_E_DEVICE, "batch events"));
  hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed);
  for (auto &g : b->groups)
    if (e == hipSuccess)
      e = launch_reset(reinterpret_cast<uint32_t *>(g.d_ctr), reinterpret_cast<unsigned long long *>(g.d_done),
                       (uint32_t)g.P.size(), b->cap);
  for (auto &g : b->groups)
    if (e == hipSuccess)
      e = launch_walk_persist(g.prec, g.sig, reinterpret_cast<const DevReq *>(g.d_reqs), (uint32_t)g.P.size(),
                              reinterpret_cast<const uint32_t *>(g.d_ws), 0u, refill_mask(ctx), g.blocks, g.threads,
                              g.lds_bytes, b->cap);
  if (e == hipSuccess) e = launch_reduce(reinterpret_cast<const NodeJob *>(b->d_jobs), (uint32_t)b->total_nodes, b->cap);
  if (e == hipSuccess && b->total_nodes)
    e = hipMemcpyAsync(b->h_out, b->d_out, b->total_nodes * sizeof(NodeOut), hipMemcpyDeviceToHost, b->cap);
  if (e == hipSuccess && n)
    e = hipMemcpyAsync(b->h_done, b->d_done_all, n * sizeof(unsigned long long), hipMemcpyDeviceToHost, b->cap);
  hipGraph_t graph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(b->cap, &graph);
  b->graph = graph;
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return bail(fail(SDD_E_DEVICE, "graph capture: %s", hipGetErrorString(e)));
  // the batch holds its workspace until destroyed: served admission counts
  // it as unavailable
  uint64_t held = Arena::round(std::max<size_t>(n, 1) * sizeof(unsigned long long)) +
                  Arena::round(std::max<uint64_t>(b->total_nodes, 1) * sizeof(NodeOut)) +
                  Arena::round(std::max<uint64_t>(b->total_nodes, 1) * sizeof(NodeJob));
  for (auto &P : b->Ps) held += pass_bytes(*P);
  for (auto &g : b->groups)
    held += Arena::round(g.P.size() * sizeof(DevReq)) + Arena::round(g.P.size() * sizeof(uint32_t)) +
            Arena::round((g.P.size() + 1) * sizeof(uint32_t));
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->held_long += held;
  }
  b->held = held;
  *out = b;
  for (uint32_t i = 0; i < n; ++i) b->Ps[i]->slot = done_index[i];
  return SDD_OK;
}

sdd_status sdd_batch_run(sdd_batch_t b, sdd_result *res) {
  if (!b) return fail(SDD_E_INVALID, "batch is NULL");
  const uint32_t n = (uint32_t)b->Ps.size();
  if (n && !res) return fail(SDD_E_INVALID, "results are NULL");
  sdd_ctx *ctx = b->ctx;
  ExecGuard ex(ctx);
  HIP_TRY(hipSetDevice(ctx->device));
  // the replay is timed as a whole (counter reset, walks, reduction, result
  // copies); the walks are all but a fraction of a percent of it
  HIP_TRY(hipEventRecord(b->ev[0], ctx->stream));
  HIP_TRY(hipGraphLaunch(b->exec, ctx->stream));
  HIP_TRY(hipEventRecord(b->ev[1], ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, b->ev[0], b->ev[1]) == hipSuccess) ctx->stats.last_walk_ms = ms;
  ctx->stats.launches += b->groups.size();
  if (!b->groups.empty()) {
    ctx->stats.last_blocks = b->groups.back().blocks;
    ctx->stats.last_threads = b->groups.back().threads;
  }
  uint64_t row = 0, steps = 0, paths = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const Prepared &P = *b->Ps[i];
    if (b->h_done[P.slot] != P.n_paths)
      return fail(SDD_E_DEVICE, "request %u: %llu of %llu paths completed", i, b->h_done[P.slot],
                  (unsigned long long)P.n_paths);
    scatter(P, b->h_out + row, &res[i]);
    for (uint32_t j = 0; j < P.pbeg.size(); ++j) steps += b->h_out[row + j].steps;
    row += P.pbeg.size();
    paths += P.n_paths;
    sdd_status st = copy_records(ctx, P, &res[i]);
    if (st != SDD_OK) return st;
  }
  ctx->stats.last_walk_steps = steps;
  ctx->stats.last_walk_paths = paths;
  return SDD_OK;
}

sdd_status sdd_batch_destroy(sdd_batch_t b) {
  if (!b) return fail(SDD_E_INVALID, "batch is NULL");
  sdd_ctx *ctx = b->ctx;
  ExecGuard ex(ctx);
  batch_free(b);
  return SDD_OK;
}

}  // extern "C"
