// HIP kernels for gfx950: the Feynman-Kac walk of the 2-D TE equation at
// interface nodes and the per-node reduction.
//
//   walk_plain     FP64, one thread per path, one launch per node (the plain
//                  form): a wave waits for its longest path.
//   walk_persist   persistent walker, FP64 or FP32-mixed: each wave owns one
//                  request at a time, claims tiles of paths with one atomic,
//                  and refills every lane whose path has exited (ballot +
//                  mbcnt rank), so lanes stay busy until the request's tiles
//                  run out.
//   reduce_nodes   deterministic FP64 reduction of each node's path records
//                  to the MC estimate, variance, covariance and SE.
//
// The arithmetic of one path is a pure function of (seed, stream, node, path)
// and the request's data, and every path writes its own record, so results
// are bitwise independent of scheduling, batch mix and launch shape.
//
// Method: Sec. 3.1 of the paper -- modified Euler-Maruyama step (Eq. 13),
// outer boundary first, Brownian-bridge hitting test (Eq. 14) on the nearer
// wall per axis, equal-kappa interface rule (phase of a step goes to the
// region of the proposed point), MC estimator with the occupation times
// folded into the phase S = sum_r (alpha_r / 2) T_r.
//
// This file is compiled with -ffp-contract=off: the FP64 walk rounds every
// operation separately (as a plain FP64 reference does); the FP32 walk asks
// for its fused multiply-adds explicitly.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sdd_device.h"

namespace sdd {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// products; the key schedule depends only on the (wave-uniform) key, so it
// runs on the scalar unit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

// ---------------------------------------------------------------------------
// Precision policies.
// ---------------------------------------------------------------------------
template <class R> struct Arith;

// FP64: the uniform (w + 1/2) 2^-32 is exact; library log/sqrt/sin/cos.
template <> struct Arith<double> {
  static __device__ __forceinline__ double u01(uint32_t w) {
    return ((double)w + 0.5) * (1.0 / 4294967296.0);
  }
  static __device__ __forceinline__ void normals(uint32_t a, uint32_t b, double &n0, double &n1) {
    const double two_pi = 6.283185307179586476925286766559;
    const double r = sqrt(-2.0 * log(u01(a)));
    const double th = two_pi * u01(b);
    n0 = r * cos(th);
    n1 = r * sin(th);
  }
  static __device__ __forceinline__ double neglog_u(uint32_t w) { return -log(u01(w)); }
  static __device__ __forceinline__ double mad(double a, double b, double c) { return c + a * b; }
};

// FP32: the uniform ((w >> 8) + 1/2) 2^-24 is exact in FP32; hardware
// transcendentals: v_log_f32 (log2), v_sqrt_f32, and v_sin/v_cos_f32 whose
// argument is in revolutions, so the angle 2 pi u needs no multiply.
template <> struct Arith<float> {
  static __device__ __forceinline__ float u01(uint32_t w) {
    return __builtin_fmaf((float)(w >> 8), 0x1p-24f, 0x1p-25f);
  }
  static __device__ __forceinline__ void normals(uint32_t a, uint32_t b, float &n0, float &n1) {
    const float m2ln2 = -1.3862943611198906f;  // -2 ln 2
    const float r = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u01(a)));
    const float ub = u01(b);
    n0 = r * __builtin_amdgcn_cosf(ub);
    n1 = r * __builtin_amdgcn_sinf(ub);
  }
  static __device__ __forceinline__ float neglog_u(uint32_t w) {
    return -0.69314718055994531f * __builtin_amdgcn_logf(u01(w));
  }
  static __device__ __forceinline__ float mad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
};

// Wave-uniform request data in registers.
template <class R> struct Uni;
template <> struct Uni<double> {
  double ylo, yhi, zlo, zhi, s, dt, thr;
  __device__ __forceinline__ void load(const DevReq &Q) {
    ylo = Q.y_lo; yhi = Q.y_hi; zlo = Q.z_lo; zhi = Q.z_hi; s = Q.s; dt = Q.dt; thr = Q.thr;
  }
};
template <> struct Uni<float> {
  float ylo, yhi, zlo, zhi, s, dt, thr;
  __device__ __forceinline__ void load(const DevReq &Q) {
    ylo = Q.fy_lo; yhi = Q.fy_hi; zlo = Q.fz_lo; zhi = Q.fz_hi; s = Q.fs; dt = Q.fdt; thr = Q.fthr;
  }
};

template <class R> __device__ __forceinline__ R creg(const DevReq &Q, int k);
template <> __device__ __forceinline__ double creg<double>(const DevReq &Q, int k) { return Q.c[k]; }
template <> __device__ __forceinline__ float creg<float>(const DevReq &Q, int k) { return Q.fc[k]; }
template <class R> __device__ __forceinline__ const R *prm(const DevReq &Q, int k);
template <> __device__ __forceinline__ const double *prm<double>(const DevReq &Q, int k) { return Q.pd[k]; }
template <> __device__ __forceinline__ const float *prm<float>(const DevReq &Q, int k) { return Q.pf[k]; }

// Phase increment of the region containing (y, z): primitives in list order,
// the first match wins, else the background (index nprims).  The loop is
// wave-uniform (scalar loads of the model); only the tests are per lane.
template <class R>
__device__ __forceinline__ R region_c(const DevReq &Q, R y, R z) {
  const int np = (int)Q.nprims;
  R c = creg<R>(Q, np);
  for (int k = np - 1; k >= 0; --k) {
    const int kind = Q.kind[k];
    const R *v = prm<R>(Q, k);
    bool in;
    if (kind == kHalfZ) {
      in = z < v[0];
    } else if (kind == kHalfY) {
      in = y < v[0];
    } else if (kind == kBox) {
      in = (y >= v[0]) && (y < v[1]) && (z >= v[2]) && (z < v[3]);
    } else {
      const R e0 = (v[2] - v[0]) * (z - v[1]) - (v[3] - v[1]) * (y - v[0]);
      const R e1 = (v[4] - v[2]) * (z - v[3]) - (v[5] - v[3]) * (y - v[2]);
      const R e2 = (v[0] - v[4]) * (z - v[5]) - (v[1] - v[5]) * (y - v[4]);
      const bool nn = (e0 >= R(0)) && (e1 >= R(0)) && (e2 >= R(0));
      const bool np_ = (e0 <= R(0)) && (e1 <= R(0)) && (e2 <= R(0));
      in = nn || np_;
    }
    c = in ? creg<R>(Q, k) : c;
  }
  return c;
}

// Walker state of one lane.
template <class R> struct Walker {
  R y, z;
  R shi, slo;   // phase S = shi + slo (slo stays 0 in FP64)
  R cc;         // phase increment of the region of the current point
  uint32_t n;   // index of the next step
  uint32_t path, node;
  uint64_t rec;
};

template <class R> __device__ __forceinline__ void add_phase(Walker<R> &W, R c);
template <> __device__ __forceinline__ void add_phase<double>(Walker<double> &W, double c) {
  W.shi = W.shi + c;
}
// Compensated FP32 (Knuth's TwoSum): shi + slo carries S to ~2^-48 relative.
template <> __device__ __forceinline__ void add_phase<float>(Walker<float> &W, float c) {
  const float s = W.shi + c;
  const float bb = s - W.shi;
  const float e = (W.shi - (s - bb)) + (c - bb);
  W.shi = s;
  W.slo = W.slo + e;
}

template <class R> struct ExitInfo {
  R f, t;
  int wall;
};

// One step of the walk.  Returns true when the step reaches the outer
// boundary (ExitInfo filled, walker state left at the last inside point);
// otherwise the proposal is accepted and its region's phase added.
template <class R>
__device__ __forceinline__ bool walk_step(const DevReq &Q, const Uni<R> &U, uint32_t k0, uint32_t k1,
                                          uint32_t ctr3, Walker<R> &W, R n0, R n1, ExitInfo<R> &X) {
  const R yn = Arith<R>::mad(U.s, n0, W.y);
  const R zn = Arith<R>::mad(U.s, n1, W.z);
  // nearer wall per axis; a tie goes to the lower wall
  const R dly = W.y - U.ylo, dhy = U.yhi - W.y;
  const bool upy = !(dly <= dhy);
  const R d0y = upy ? dhy : dly;
  const R d1y = upy ? (U.yhi - yn) : (yn - U.ylo);
  const R dlz = W.z - U.zlo, dhz = U.zhi - W.z;
  const bool upz = !(dlz <= dhz);
  const R d0z = upz ? dhz : dlz;
  const R d1z = upz ? (U.zhi - zn) : (zn - U.zlo);
  const bool cy = d1y <= R(0);
  const bool cz = d1z <= R(0);
  const R qy = (R(2) * d0y) * d1y;
  const R qz = (R(2) * d0z) * d1z;
  bool hy = cy, hz = cz;
  R fy = R(0), fz = R(0);
  // Same side: the bridge can only have hit when 2 d0 d1 <= dt (-log U) and
  // -log U <= 22.87 for every U this generator makes, so U is drawn only
  // below the threshold thr = 22.9 dt.
  const bool ny = !cy && (qy <= U.thr);
  const bool nz = !cz && (qz <= U.thr);
  if (ny || nz) {
    const uint4 b = philox10(W.n, W.path, W.node, ctr3 + 1u, k0, k1);
    if (ny) {
      const R L = Arith<R>::neglog_u(b.x);
      if (qy <= U.dt * L) { hy = true; fy = qy / (U.dt * L); }
    }
    if (nz) {
      const R L = Arith<R>::neglog_u(b.y);
      if (qz <= U.dt * L) { hz = true; fz = qz / (U.dt * L); }
    }
  }
  if (hy || hz) {
    if (cy) fy = d0y / (d0y - d1y);
    if (cz) fz = d0z / (d0z - d1z);
    const bool usey = hy && (!hz || fy <= fz);
    if (usey) {
      X.f = fy;
      X.wall = upy ? 1 : 3;
      R t = W.z + fy * (zn - W.z);
      t = t < U.zlo ? U.zlo : t;
      t = t > U.zhi ? U.zhi : t;
      X.t = t;
    } else {
      X.f = fz;
      X.wall = upz ? 2 : 0;
      R t = W.y + fz * (yn - W.y);
      t = t < U.ylo ? U.ylo : t;
      t = t > U.yhi ? U.yhi : t;
      X.t = t;
    }
    return true;
  }
  const R c = region_c<R>(Q, yn, zn);
  add_phase<R>(W, c);
  W.cc = c;
  W.y = yn;
  W.z = zn;
  return false;
}

// The weight g(X_tau) exp(-i S) of a finished path, in FP64.
template <class R>
__device__ __forceinline__ PathRec finish_path(const DevReq &Q, const Walker<R> &W, const ExitInfo<R> &X) {
  double S;
  if constexpr (sizeof(R) == 8) {
    S = (double)W.shi + (double)(W.cc * X.f);
  } else {
    S = ((double)W.shi + (double)W.slo) + (double)(W.cc * X.f);
  }
  const int wall = X.wall;
  const bool along_y = (wall == 0) || (wall == 2);
  const double t0 = along_y ? Q.y_lo : Q.z_lo;
  const double t1 = along_y ? Q.y_hi : Q.z_hi;
  const int M = (int)Q.M;
  const double h = (t1 - t0) / (double)M;
  const double u = ((double)X.t - t0) / h;
  int i = (int)floor(u);
  i = i < 0 ? 0 : i;
  i = i > M - 1 ? M - 1 : i;
  const double lam = u - (double)i;
  const double *gw = Q.g + (size_t)wall * (size_t)(M + 1) * 2;
  const double2 ga = *reinterpret_cast<const double2 *>(gw + 2 * i);
  const double2 gb = *reinterpret_cast<const double2 *>(gw + 2 * i + 2);
  const double gre = (1.0 - lam) * ga.x + lam * gb.x;
  const double gim = (1.0 - lam) * ga.y + lam * gb.y;
  const double cs = cos(S), sn = sin(S);
  PathRec r;
  r.w_re = gre * cs + gim * sn;
  r.w_im = gim * cs - gre * sn;
  r.tau = ((double)W.n + (double)X.f) * Q.dt;
  r.steps = W.n + 1u;
  r.wall = wall;
  return r;
}

__device__ __forceinline__ PathRec unfinished_rec(uint32_t steps) {
  PathRec r;
  r.w_re = 0.0;
  r.w_im = 0.0;
  r.tau = -1.0;
  r.steps = steps;
  r.wall = -1;
  return r;
}

template <class R>
__device__ __forceinline__ void start_walker(const DevReq &Q, Walker<R> &W, uint32_t node, uint32_t path,
                                             uint64_t rec) {
  const double2 p = *reinterpret_cast<const double2 *>(Q.nodes + 2 * (size_t)node);
  W.y = (R)p.x;
  W.z = (R)p.y;
  W.shi = R(0);
  W.slo = R(0);
  W.n = 0;
  W.path = path;
  W.node = node;
  W.rec = rec;
  W.cc = region_c<R>(Q, W.y, W.z);
}

// ---------------------------------------------------------------------------
// Plain FP64 walker: one thread walks one path to its end.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) walk_plain(const DevReq *__restrict__ reqs, uint32_t node,
                                                  uint32_t p0, uint32_t count, uint64_t rec0) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= count) return;
  const DevReq &Q = reqs[0];
  Uni<double> U;
  U.load(Q);
  const uint32_t k0 = Q.key0, k1 = Q.key1, ctr3 = Q.ctr3, max_steps = Q.max_steps;
  Walker<double> W;
  start_walker<double>(Q, W, node, p0 + tid, rec0 + tid);
  ExitInfo<double> X;
  while (W.n < max_steps) {
    const uint4 w = philox10(W.n >> 1, W.path, W.node, ctr3, k0, k1);
    double a0, a1, b0, b1;
    Arith<double>::normals(w.x, w.y, a0, a1);
    Arith<double>::normals(w.z, w.w, b0, b1);
    if (walk_step<double>(Q, U, k0, k1, ctr3, W, a0, a1, X)) {
      Q.recs[W.rec] = finish_path<double>(Q, W, X);
      return;
    }
    W.n += 1u;
    if (W.n >= max_steps) break;
    if (walk_step<double>(Q, U, k0, k1, ctr3, W, b0, b1, X)) {
      Q.recs[W.rec] = finish_path<double>(Q, W, X);
      return;
    }
    W.n += 1u;
  }
  Q.recs[W.rec] = unfinished_rec(max_steps);
}

// ---------------------------------------------------------------------------
// Persistent walker.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint32_t pick_request(const DevReq *__restrict__ reqs, uint32_t n_req) {
  // the request with the most unclaimed tiles (ties: lowest index)
  uint32_t best = kNoRequest, best_left = 0;
  for (uint32_t r = 0; r < n_req; ++r) {
    const uint32_t taken = uni(__hip_atomic_load(reqs[r].tile_counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const uint32_t nt = reqs[r].n_tiles;
    const uint32_t left = taken < nt ? nt - taken : 0u;
    if (left > best_left) { best_left = left; best = r; }
  }
  return best;
}

template <class R>
__device__ __forceinline__ void run_request(const DevReq &Q) {
  const uint32_t lane = __lane_id();
  Uni<R> U;
  U.load(Q);
  const uint32_t k0 = Q.key0, k1 = Q.key1, ctr3 = Q.ctr3, max_steps = Q.max_steps;
  const uint32_t n_tiles = Q.n_tiles;

  Walker<R> W;
  W.n = 0; W.path = 0; W.node = 0; W.rec = 0;
  W.y = R(0); W.z = R(0); W.shi = R(0); W.slo = R(0); W.cc = R(0);
  bool active = false;

  // wave-uniform tile cursor
  uint32_t t_node = 0, t_p0 = 0, t_next = 0, t_end = 0;
  uint64_t t_rec0 = 0;
  bool exhausted = false;
  uint32_t finished = 0;   // paths this wave completed (wave-uniform)

  for (;;) {
    // refill free lanes in rank order from the wave's tile, claiming tiles
    const uint64_t freemask = __ballot(!active);
    if (freemask != 0ull && !exhausted) {
      const uint32_t nfree = (uint32_t)__popcll(freemask);
      const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(freemask >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)freemask, 0u));
      uint32_t given = 0;
      while (given < nfree) {
        if (t_next == t_end) {
          uint32_t t = 0;
          if (lane == 0) t = atomicAdd(Q.tile_counter, 1u);
          t = uni(t);
          if (t >= n_tiles) { exhausted = true; break; }
          const DevTile T = Q.tiles[t];
          t_node = uni(T.node);
          t_p0 = uni(T.p0);
          t_next = t_p0;
          t_end = t_p0 + uni(T.count);
          t_rec0 = ((uint64_t)uni((uint32_t)(T.rec0 >> 32)) << 32) | uni((uint32_t)T.rec0);
        }
        const uint32_t take = min(t_end - t_next, nfree - given);
        if (!active && rank >= given && rank < given + take) {
          const uint32_t p = t_next + (rank - given);
          start_walker<R>(Q, W, t_node, p, t_rec0 + (p - t_p0));
          active = true;
        }
        t_next += take;
        given += take;
      }
    }
    const uint64_t freemask_after_refill = __ballot(!active);
    if (freemask_after_refill == ~0ull) break;

    if (active) {
      // two steps per Philox call: words 0,1 for step n (even), 2,3 for n+1
      const uint4 w = philox10(W.n >> 1, W.path, W.node, ctr3, k0, k1);
      R a0, a1, b0, b1;
      Arith<R>::normals(w.x, w.y, a0, a1);
      Arith<R>::normals(w.z, w.w, b0, b1);
      ExitInfo<R> X;
      bool ex = walk_step<R>(Q, U, k0, k1, ctr3, W, a0, a1, X);
      if (!ex) {
        W.n += 1u;
        if (W.n < max_steps) {
          ex = walk_step<R>(Q, U, k0, k1, ctr3, W, b0, b1, X);
          if (!ex) W.n += 1u;
        }
      }
      if (ex) {
        Q.recs[W.rec] = finish_path<R>(Q, W, X);
        active = false;
      } else if (W.n >= max_steps) {
        Q.recs[W.rec] = unfinished_rec(max_steps);
        active = false;
      }
    }
    finished += (uint32_t)__popcll(__ballot(!active)) - (uint32_t)__popcll(freemask_after_refill);
  }
  if (lane == 0) atomicAdd(Q.done_counter, (unsigned long long)finished);
}

__global__ void __launch_bounds__(256) walk_persist(const DevReq *__restrict__ reqs, uint32_t n_req,
                                                    const uint32_t *__restrict__ wave_start) {
  const uint32_t wid = uni((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  // initial request: waves are shared out in proportion to each request's work
  uint32_t r = kNoRequest;
  for (uint32_t i = 0; i < n_req; ++i)
    if (wid >= wave_start[i] && wid < wave_start[i + 1]) r = i;
  r = uni(r);
  // Each visit either claims a tile or finds the request's tiles exhausted,
  // after which pick_request never returns it again: the loop ends once every
  // tile of every request has been claimed.
  while (r != kNoRequest) {
    const DevReq &Q = reqs[r];
    if (Q.precision == 0u) run_request<double>(Q);
    else run_request<float>(Q);
    r = pick_request(reqs, n_req);
  }
}

// ---------------------------------------------------------------------------
// Deterministic per-node reduction (fixed order: strided per-thread sums,
// butterfly within the wave, waves in index order).
// ---------------------------------------------------------------------------
constexpr int kRedThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double (*lds)[K]) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[w][k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int i = 0; i < kRedThreads / 64; ++i) s += lds[i][k];
    v[k] = s;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kRedThreads) reduce_nodes(const NodeJob *__restrict__ jobs) {
  __shared__ double lds[kRedThreads / 64][4];
  __shared__ unsigned long long ldsu[kRedThreads / 64][3];
  const NodeJob J = jobs[blockIdx.x];
  const int tid = threadIdx.x;
  const uint64_t count = J.count0 + J.count1;
  auto rec = [&](uint64_t i) { return i < J.count0 ? J.recs0[i] : J.recs1[i - J.count0]; };
  double s[4] = {0.0, 0.0, 0.0, 0.0};  // sum re, sum im, sum tau, (unused)
  unsigned long long cnt[3] = {0ull, 0ull, 0ull};  // done, unfinished, steps
  for (uint64_t i = tid; i < count; i += kRedThreads) {
    const PathRec r = rec(i);
    cnt[2] += r.steps;
    if (r.wall < 0) { cnt[1] += 1ull; continue; }
    cnt[0] += 1ull;
    s[0] += r.w_re;
    s[1] += r.w_im;
    s[2] += r.tau;
  }
  block_sum<4>(s, lds);
  {
    const int w = tid >> 6, lane = tid & 63;
    for (int k = 0; k < 3; ++k) cnt[k] = wave_sum_u64(cnt[k]);
    if (lane == 0) for (int k = 0; k < 3; ++k) ldsu[w][k] = cnt[k];
    __syncthreads();
    for (int k = 0; k < 3; ++k) {
      unsigned long long t = 0;
      for (int i = 0; i < kRedThreads / 64; ++i) t += ldsu[i][k];
      cnt[k] = t;
    }
  }
  const double N = (double)cnt[0];
  const double mre = s[0] / N, mim = s[1] / N;
  double q[4] = {0.0, 0.0, 0.0, 0.0};  // (re-m)^2, (im-m)^2, (re-m)(im-m)
  for (uint64_t i = tid; i < count; i += kRedThreads) {
    const PathRec r = rec(i);
    if (r.wall < 0) continue;
    const double dr = r.w_re - mre, di = r.w_im - mim;
    q[0] += dr * dr;
    q[1] += di * di;
    q[2] += dr * di;
  }
  block_sum<4>(q, lds);
  if (tid == 0) {
    NodeOut o;
    o.mean_re = mre;
    o.mean_im = mim;
    o.mean_exit_time = s[2] / N;
    o.var_re = q[0] / (N - 1.0);
    o.var_im = q[1] / (N - 1.0);
    o.cov = q[2] / (N - 1.0);
    o.se_re = sqrt(o.var_re / N);
    o.se_im = sqrt(o.var_im / N);
    o.se = sqrt((o.var_re + o.var_im) / N);
    o.paths_done = cnt[0];
    o.unfinished = cnt[1];
    o.steps = cnt[2];
    *J.out = o;
  }
}

// Sets every request's claim counter and done counter to zero (a kernel, so
// the launch sequence can be captured and replayed as a graph).
__global__ void reset_counters(uint32_t *tile_counters, unsigned long long *done, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    tile_counters[i] = 0u;
    done[i] = 0ull;
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
hipError_t launch_walk_plain(const DevReq *req_dev, uint32_t node, uint32_t p0, uint32_t count, uint64_t rec0,
                             hipStream_t st) {
  if (count == 0) return hipSuccess;
  const uint32_t blocks = (count + 255u) / 256u;
  hipLaunchKernelGGL(walk_plain, dim3(blocks), dim3(256), 0, st, req_dev, node, p0, count, rec0);
  return hipGetLastError();
}

hipError_t launch_walk_persist(const DevReq *reqs_dev, uint32_t n_req, const uint32_t *wave_start_dev,
                               uint32_t blocks, uint32_t threads, hipStream_t st) {
  hipLaunchKernelGGL(walk_persist, dim3(blocks), dim3(threads), 0, st, reqs_dev, n_req, wave_start_dev);
  return hipGetLastError();
}

hipError_t launch_reduce(const NodeJob *jobs_dev, uint32_t n_jobs, hipStream_t st) {
  if (n_jobs == 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_nodes, dim3(n_jobs), dim3(kRedThreads), 0, st, jobs_dev);
  return hipGetLastError();
}

int persist_blocks_per_cu(uint32_t threads) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, walk_persist, (int)threads, 0) != hipSuccess) return 0;
  return nb;
}

hipError_t launch_reset(uint32_t *tile_counters, unsigned long long *done, uint32_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(reset_counters, dim3((n + 255u) / 256u), dim3(256), 0, st, tile_counters, done, n);
  return hipGetLastError();
}

}  // namespace sdd
