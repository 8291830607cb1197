// HIP kernels for gfx950: the Feynman-Kac walk of the 2-D TE equation at
// interface nodes and the per-node reduction.
//
//   walk_plain        FP64, one thread per path, one launch per node (the
//                     plain form): a wave waits for its longest path.
//   walk_persist_f64  persistent walker, FP64: the arithmetic of a plain
//                     FP64 reference on the same streams (the uniforms' log
//                     and full-turn sine/cosine from sdd_math64.h, within
//                     2 ulp of the exact values).
//   walk_persist_f32  persistent walker, FP32-mixed: coordinates relative to
//                     the domain centre, a conservative exit screen per
//                     pair of steps (the least distance of three points
//                     to the walls), the phase as exact per-region step
//                     counts or a 64-bit fixed-point sum; weight and
//                     reduction in FP64.
//   reduce_nodes      deterministic FP64 reduction of each node's path records
//                     to the MC estimate, variance, covariance and SE.
//
// Persistent walkers: each wave owns one request at a time, claims tiles of
// paths with one atomic and refills every lane whose path has exited (ballot
// + mbcnt rank), so lanes stay busy until the request's tiles run out.  The
// request data sit in SGPRs, walker state in VGPRs.  The region lookup is
// specialised per model signature (a wave-uniform dispatch), with the
// model's parameters hoisted into registers once per request.
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

#include <mutex>

#include "sdd_device.h"
#include "sdd_rng.h"

namespace sdd {

// ---------------------------------------------------------------------------
// Static scratch of sdd_solve_noalloc: every device buffer such a solve needs
// beyond its inputs and outputs (descriptor, counters, tables, nodes, sigma
// grid, tiles, path records, reduction jobs and rows) is carved from this
// one array, so that call allocates nothing.  Each GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never passes the array's name to a kernel or a copy: it uses the address
// hipGetSymbolAddress returns on each device, taken once per device with that
// device current (scratch_init, called by sdd_create).
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxScratchDevices] = {};
static std::mutex g_scratch_use[kMaxScratchDevices];

// The scratch address on `device`, which must be the current device.
hipError_t scratch_init(int device, void **out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

size_t scratch_bytes() { return kScratchBytes; }

// Calls on one device share its scratch: each holds this lock until its
// results are on the host.
std::mutex &scratch_lock(int device) { return g_scratch_use[device]; }

template <class R> struct ExitInfo {
  R f, t;     // fraction of the last step; tangential coordinate of the exit
  int wall;   // 0 top, 1 right, 2 bottom, 3 left
};

// ---------------------------------------------------------------------------
// Region lookup: the phase increment c of the region containing a point.
// Primitives in list order, the first match wins, else the background.
// ---------------------------------------------------------------------------

// Closed triangle.  FP64: every edge function from the vertices >= 0 or
// every one <= 0 (either orientation; the plain definition).  FP32: edge k
// from its (A, B, C), e = fma(A, y, fma(B, z, C)), the expression the sigma
// grid's lines use, with the edges oriented by the host so that the interior
// is e >= 0 on all three (the three edge functions sum to twice the signed
// area, so no point of a triangle of positive area has all three below zero
// beyond their rounding).
template <class R>
__device__ __forceinline__ bool tri_in(const R *v, R y, R z) {
  if constexpr (sizeof(R) == 8) {
    const R e0 = (v[2] - v[0]) * (z - v[1]) - (v[3] - v[1]) * (y - v[0]);
    const R e1 = (v[4] - v[2]) * (z - v[3]) - (v[5] - v[3]) * (y - v[2]);
    const R e2 = (v[0] - v[4]) * (z - v[5]) - (v[1] - v[5]) * (y - v[4]);
    return ((e0 >= R(0)) & (e1 >= R(0)) & (e2 >= R(0))) | ((e0 <= R(0)) & (e1 <= R(0)) & (e2 <= R(0)));
  } else {
    const R e0 = __builtin_fmaf(v[0], y, __builtin_fmaf(v[1], z, v[2]));
    const R e1 = __builtin_fmaf(v[3], y, __builtin_fmaf(v[4], z, v[5]));
    const R e2 = __builtin_fmaf(v[6], y, __builtin_fmaf(v[7], z, v[8]));
    return fminf(fminf(e0, e1), e2) >= 0.f;
  }
}

// Generic: loop over the primitives (kinds and parameters wave-uniform);
// cv[k] is the value of region k (an FP64 rate, or a fixed-point increment).
template <class R, int STRIDE, class V>
__device__ __forceinline__ V region_c_generic(int np, const int32_t *kind, const R *prm, const V *cv, R y, R z) {
  V c = cv[np];
  for (int k = np - 1; k >= 0; --k) {
    const int kd = kind[k];
    const R *v = prm + k * STRIDE;
    bool in;
    if (kd == kHalfZ) {
      in = z < v[0];
    } else if (kd == kHalfY) {
      in = y < v[0];
    } else if (kd == kBox) {
      in = (y >= v[0]) & (y < v[1]) & (z >= v[2]) & (z < v[3]);
    } else {
      in = tri_in<R>(v, y, z);
    }
    c = in ? cv[k] : c;
  }
  return c;
}

// FP64 lookup, exactly the plain definition (absolute coordinates).  The
// specialised signatures hold the same primitives' parameters in registers.
template <int SIG> struct Reg64 {
  double cb, c0, c1;
  double v[6];   // parameters of primitive 1 (HALF_Y / BOX / TRIANGLE)
  double z0;     // primitive 0: air above z0
  __device__ __forceinline__ void load(const DevReq &Q) {
    const int np = (int)Q.nprims;
    cb = unid(Q.c[np]);
    if constexpr (SIG != kSigNone && SIG != kSigGeneric) {
      c0 = unid(Q.c[0]);
      z0 = unid(Q.pd[0][0]);
    }
    if constexpr (SIG == kSigZY || SIG == kSigZBox || SIG == kSigZTri) {
      c1 = unid(Q.c[1]);
#pragma unroll
      for (int i = 0; i < 6; ++i) v[i] = unid(Q.pd[1][i]);
    }
  }
  // The operands go through readfirstlane (free on uniform values) so that
  // each select is between values, never a load through a selected pointer
  // (which would keep the request data in scratch memory).
  __device__ __forceinline__ double eval(const DevReq &Q, double y, double z) const {
    if constexpr (SIG == kSigNone) {
      return unid(cb);
    } else if constexpr (SIG == kSigZ) {
      return z < unid(z0) ? unid(c0) : unid(cb);
    } else if constexpr (SIG == kSigZY) {
      const double c = y < unid(v[0]) ? unid(c1) : unid(cb);
      return z < unid(z0) ? unid(c0) : c;
    } else if constexpr (SIG == kSigZBox) {
      const bool in = (y >= unid(v[0])) & (y < unid(v[1])) & (z >= unid(v[2])) & (z < unid(v[3]));
      const double c = in ? unid(c1) : unid(cb);
      return z < unid(z0) ? unid(c0) : c;
    } else if constexpr (SIG == kSigZTri) {
      const double v0 = unid(v[0]), v1 = unid(v[1]), v2 = unid(v[2]), v3 = unid(v[3]), v4 = unid(v[4]),
                   v5 = unid(v[5]);
      const double e0 = (v2 - v0) * (z - v1) - (v3 - v1) * (y - v0);
      const double e1 = (v4 - v2) * (z - v3) - (v5 - v3) * (y - v2);
      const double e2 = (v0 - v4) * (z - v5) - (v1 - v5) * (y - v4);
      const bool in = ((e0 >= 0.0) & (e1 >= 0.0) & (e2 >= 0.0)) | ((e0 <= 0.0) & (e1 <= 0.0) & (e2 <= 0.0));
      const double c = in ? unid(c1) : unid(cb);
      return z < unid(z0) ? unid(c0) : c;
    } else {
      return region_c_generic<double, 6>((int)Q.nprims, Q.kind, &Q.pd[0][0], Q.c, y, z);
    }
  }
};

// Index of the first primitive containing (y, z), or np (background).
template <class R, int STRIDE>
__device__ __forceinline__ int region_index_generic(int np, const int32_t *kind, const R *prm, R y, R z) {
  int idx = np;
  for (int k = np - 1; k >= 0; --k) {
    const int kd = kind[k];
    const R *v = prm + k * STRIDE;
    bool in;
    if (kd == kHalfZ) {
      in = z < v[0];
    } else if (kd == kHalfY) {
      in = y < v[0];
    } else if (kd == kBox) {
      in = (y >= v[0]) & (y < v[1]) & (z >= v[2]) & (z < v[3]);
    } else {
      in = tri_in<R>(v, y, z);
    }
    idx = in ? k : idx;
  }
  return idx;
}

// The LDS form of the sigma grid (kSigGenericLds): one class byte per cell,
// then the class table (SigmaCells), staged by each block at the start of the
// launch.
extern __shared__ __attribute__((aligned(16))) uint8_t g_lds[];

// The primitive loop for the sigma grid's few cells crossed by more than two
// boundaries, out of line so that its registers stay out of the walker loop.
__device__ __noinline__ uint32_t loop_fallback(const DevReq &Q, float a, float b) {
  return region_c_generic<float, kPfStride>((int)Q.nprims, Q.kind, &Q.pf[0][0], Q.cfx, a, b);
}

// FP32 region tests in centred coordinates; the triangle as three linear
// forms.  The specialised signatures have at most three regions: primitive 0
// (air above z0), primitive 1 (half-plane, box or triangle) and the
// background.  Their walkers count full steps per region instead of summing
// phase increments: the phase of n full steps is then exactly
// c0 n0 + c1 n1 + cb (n - n0 - n1), formed in FP64 when the path exits.  The
// generic signature adds each step's fixed-point increment (the region's
// phase in units of 2^-phase_shift, an integer below 2^31) to a 64-bit sum,
// which is exact: only the one rounding of each region's phase to an integer
// remains, below 2^-32 of the largest per step.
template <int SIG> struct Reg32 {
  static constexpr bool kGeneric = SIG == kSigGeneric || SIG == kSigGenericLds;
  static constexpr bool kCounted = !kGeneric;
  float p[10];
  // generic signature: the sigma grid
  const SigmaCell *grid, *grid_ext;
  uint32_t gy, lds_table;
  float gsy, goy, gsz, goz, gmy, gmz;
  __device__ __forceinline__ void load(const DevReq &Q) {
    if constexpr (kGeneric) {
      grid = Q.grid;
      grid_ext = Q.grid_ext;
      gy = Q.gy;
      gsy = Q.gsy; goy = Q.goy; gsz = Q.gsz; goz = Q.goz;
      gmy = Q.gmy; gmz = Q.gmz;
      lds_table = Q.lds_table;
    }
    if constexpr (SIG != kSigNone && !kGeneric) p[0] = unif(Q.sigp[0]);
    if constexpr (SIG == kSigZY || SIG == kSigZBox || SIG == kSigZTri) {
#pragma unroll
      for (int i = 1; i < 10; ++i) p[i] = unif(Q.sigp[i]);
    }
  }
  // region index: 0, 1, or 2 for the background (generic: its own numbering,
  // np for the background)
  __device__ __forceinline__ bool in_prim1(float a, float b) const {
    if constexpr (SIG == kSigZY) {
      return a < unif(p[1]);
    } else if constexpr (SIG == kSigZBox) {
      return (a >= unif(p[1])) & (a < unif(p[2])) & (b >= unif(p[3])) & (b < unif(p[4]));
    } else if constexpr (SIG == kSigZTri) {
      float q[10];
#pragma unroll
      for (int i = 1; i < 10; ++i) q[i] = unif(p[i]);
      const float e0 = __builtin_fmaf(q[1], a, __builtin_fmaf(q[2], b, q[3]));
      const float e1 = __builtin_fmaf(q[4], a, __builtin_fmaf(q[5], b, q[6]));
      const float e2 = __builtin_fmaf(q[7], a, __builtin_fmaf(q[8], b, q[9]));
      return fminf(fminf(e0, e1), e2) >= 0.f;   // edges oriented: the interior is e >= 0
    } else {
      return false;
    }
  }
  __device__ __forceinline__ int index(const DevReq &Q, float a, float b) const {
    if constexpr (SIG == kSigNone) {
      return 2;
    } else if constexpr (kGeneric) {
      return region_index_generic<float, kPfStride>((int)Q.nprims, Q.kind, &Q.pf[0][0], a, b);
    } else {
      if (b < unif(p[0])) return 0;
      return in_prim1(a, b) ? 1 : 2;
    }
  }
  // one full step ending at (a, b): add it to its region's count (every
  // operand read and every test made before the adds, so that each add is
  // one add-with-carry on the test's lane mask)
  // The counts are g = steps outside primitive 0 (below the air) and
  // m = those of them inside primitive 1.
  __device__ __forceinline__ void count(float a, float b, uint32_t &g, uint32_t &m) const {
    if constexpr (SIG != kSigNone && !kGeneric) {
      const float z0 = unif(p[0]);
      const bool ground = b >= z0;
      if constexpr (SIG != kSigZ) {
        const bool in1 = in_prim1(a, b);
        m += (uint32_t)(in1 & ground);
      }
      g += (uint32_t)ground;
    }
  }
  // FP64 phase rate of region index k (specialised signatures)
  __device__ __forceinline__ double rate(const DevReq &Q, int k) const {
    return k == 2 ? Q.c[Q.nprims] : Q.c[k];
  }
  // phase of n full steps from the counts g, m
  __device__ __forceinline__ double phase(const DevReq &Q, uint32_t g, uint32_t m, uint32_t n) const {
    const double cb = unid(Q.c[Q.nprims]);
    if constexpr (SIG == kSigNone) {
      return cb * (double)n;
    } else if constexpr (SIG == kSigZ) {
      return unid(Q.c[0]) * (double)(n - g) + cb * (double)g;
    } else {
      return (unid(Q.c[0]) * (double)(n - g) + unid(Q.c[1]) * (double)m) + cb * (double)(g - m);
    }
  }
  // generic signature: the fixed-point increment of the region containing
  // (a, b).  With the sigma grid: one cell read and one edge function (a
  // second line in cells crossed by two boundaries, the primitive loop in
  // cells crossed by more); the same
  // region as the loop for every point (the host classifies cells with
  // margins for the FP32 rounding of the cell index and of the edge
  // functions).  The cell comes from LDS (kSigGenericLds: a class byte, then
  // the class's SigmaCell) or from the global grid.
  __device__ __forceinline__ uint32_t inc32(const DevReq &Q, float a, float b) const {
    if constexpr (SIG == kSigGeneric) {
      if (grid == nullptr) return region_c_generic<float, kPfStride>((int)Q.nprims, Q.kind, &Q.pf[0][0], Q.cfx, a, b);
    }
    // cell (trunc(a gsy + goy), trunc(b gsz + goz)) clamped to the grid:
    // clamping in FP32 before the truncation gives the same cell
    const uint32_t i = (uint32_t)__builtin_amdgcn_fmed3f(__builtin_fmaf(a, gsy, goy), 0.f, gmy);
    const uint32_t j = (uint32_t)__builtin_amdgcn_fmed3f(__builtin_fmaf(b, gsz, goz), 0.f, gmz);
    const uint32_t cell = __umul24(j, gy) + i;
    uint32_t inc_ge, inc_lt, xi;
    float A, B, C;
    if constexpr (SIG == kSigGenericLds) {
      // the class byte sits at the cell's own offset; the class at lds_table
      const uint32_t cls = g_lds[cell];
      const uint8_t *ce = g_lds + lds_table + cls * (uint32_t)sizeof(SigmaCell);
      const uint4 h0 = *reinterpret_cast<const uint4 *>(ce);
      const uint2 h1 = *reinterpret_cast<const uint2 *>(ce + 16);
      inc_ge = h0.x; inc_lt = h0.y;
      A = __builtin_bit_cast(float, h0.z); B = __builtin_bit_cast(float, h0.w);
      C = __builtin_bit_cast(float, h1.x); xi = h1.y;
    } else {
      // the cell's 24 bytes in flight together, through the global address
      // space (one memory latency per step)
      typedef const __attribute__((address_space(1))) uint32_t *gptr;
      const gptr w = (gptr)(grid + cell);
      inc_ge = w[0]; inc_lt = w[1];
      A = __builtin_bit_cast(float, w[2]); B = __builtin_bit_cast(float, w[3]);
      C = __builtin_bit_cast(float, w[4]); xi = w[5];
    }
    const float e = __builtin_fmaf(A, a, __builtin_fmaf(B, b, C));
    uint32_t c = e >= 0.f ? inc_ge : inc_lt;
    if (inc_ge >= kCellTwo) {   // a few cells: two lines, or the primitive loop
      if (inc_ge < kCellLoop) {
        const SigmaCell *X;
        if constexpr (SIG == kSigGenericLds)
          X = reinterpret_cast<const SigmaCell *>(g_lds + lds_table) + xi;
        else X = grid_ext + xi;
        const float e2 = __builtin_fmaf(X->A, a, __builtin_fmaf(X->B, b, X->C));
        if (e2 >= 0.f) c = e >= 0.f ? X->inc_ge : X->inc_lt;
        else c = e >= 0.f ? (inc_ge & ~kCellFlags) : inc_lt;
      } else {
        c = loop_fallback(Q, a, b);
      }
    }
    return c;
  }
};

// The weight g(X_tau) exp(-i S) of a finished path, in FP64, from the exit
// wall, the tangential coordinate t (absolute) and the phase S; g is the
// wall's table, linear between its M + 1 equispaced samples.
__device__ __forceinline__ void weight_tab(const double *g, int M, double y_lo, double y_hi, double z_lo, double z_hi,
                                           int wall, double t, double S, double &wre, double &wim) {
  double gre, gim;
  g_table(g, M, y_lo, y_hi, z_lo, z_hi, wall, t, gre, gim);
  const double cs = cos(S), sn = sin(S);
  wre = gre * cs + gim * sn;
  wim = gim * cs - gre * sn;
}

__device__ __forceinline__ void weight(const DevReq &Q, int wall, double t, double S, double &wre, double &wim) {
  weight_tab(Q.g, (int)Q.M, Q.y_lo, Q.y_hi, Q.z_lo, Q.z_hi, wall, t, S, wre, wim);
}

// Record of a finished path: its weight, or (multi-frequency requests) its
// phase and tangential exit coordinate.
__device__ __forceinline__ void finish_weight(const DevReq &Q, int wall, double t, double S, PathRec &r) {
  if (Q.fanout) {
    r.w_re = S;
    r.w_im = t;
  } else {
    weight(Q, wall, t, S, r.w_re, r.w_im);
  }
}

// finish_weight called out of line, for the walkers that hold many values
// across their loop (the FP64 walks, the generic signatures): inlined, the
// table lookup and the FP64 sine and cosine of the phase keep their constants
// and pointers live in scalar registers through the loop, which pushes loop
// values into spill slots.  Arguments and result by value (no stack copy).
__device__ __noinline__ double2 finish_weight_outline(const DevReq &Q, int wall, double t, double S) {
  PathRec r;
  finish_weight(Q, wall, t, S, r);
  return make_double2(r.w_re, r.w_im);
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

// ===========================================================================
// FP64 walk: absolute coordinates, every decision exactly as the plain
// definition takes it.
// ===========================================================================
struct W64 {
  double y, z, S, cc;   // position, phase, phase rate of the current region
  double dy, dz;        // distance of the position to its nearer wall, per axis
  uint32_t n, path, node;
  uint64_t rec;
  uint64_t P;           // M0 * (n / 2): counter product of the next normal pair
  PhiloxPath pp;
};

template <int SIG> struct U64 {
  double ylo, yhi, zlo, zhi, s, dt, thr, thr0;
  uint32_t k0, k1, ctr3, max_steps;
  Reg64<SIG> reg;
  __device__ __forceinline__ void load(const DevReq &Q) {
    ylo = Q.y_lo; yhi = Q.y_hi; zlo = Q.z_lo; zhi = Q.z_hi; s = Q.s; dt = Q.dt; thr = Q.thr;
    thr0 = thr > 0.0 ? thr : 0.0;
    k0 = Q.key0; k1 = Q.key1; ctr3 = Q.ctr3; max_steps = Q.max_steps;
    reg.load(Q);
  }
};

template <int SIG>
__device__ __forceinline__ void start64(const DevReq &Q, const U64<SIG> &U, W64 &W, uint32_t node, uint32_t path,
                                        uint64_t rec) {
  const double2 p = *reinterpret_cast<const double2 *>(Q.nodes + 2 * (size_t)node);
  W.y = p.x;
  W.z = p.y;
  W.S = 0.0;
  W.n = 0;
  W.path = path;
  W.node = node;
  W.rec = rec;
  W.P = 0;
  W.pp = philox_path(path, node, U.k0);
  W.cc = U.reg.eval(Q, W.y, W.z);
  W.dy = fmin(W.y - U.ylo, U.yhi - W.y);
  W.dz = fmin(W.z - U.zlo, U.zhi - W.z);
}

// The exact exit logic of one step from (W.y, W.z) to (yn, zn): true when
// the step reaches the outer boundary (recorded in X).
template <int SIG>
__device__ __forceinline__ bool exit64(const U64<SIG> &U, const W64 &W, double yn, double zn, ExitInfo<double> &X) {
  // nearer wall per axis; a tie goes to the lower wall
  const double dly = W.y - U.ylo, dhy = U.yhi - W.y;
  const bool upy = !(dly <= dhy);
  const double d0y = upy ? dhy : dly;
  const double d1y = upy ? (U.yhi - yn) : (yn - U.ylo);
  const double dlz = W.z - U.zlo, dhz = U.zhi - W.z;
  const bool upz = !(dlz <= dhz);
  const double d0z = upz ? dhz : dlz;
  const double d1z = upz ? (U.zhi - zn) : (zn - U.zlo);
  const bool cy = d1y <= 0.0;
  const bool cz = d1z <= 0.0;
  const double qy = (2.0 * d0y) * d1y;
  const double qz = (2.0 * d0z) * d1z;
  bool hy = cy, hz = cz;
  double fy = 0.0, fz = 0.0;
  // Same side: the bridge can only have hit when 2 d0 d1 <= dt (-log U) and
  // -log U <= 22.87 for every U made here, so U is drawn only when
  // 2 d0 d1 <= 22.9 dt.
  const bool ny = !cy && (qy <= U.thr);
  const bool nz = !cz && (qz <= U.thr);
  if (ny || nz) {
    const uint64_t Pn = (W.P << 1) + ((W.n & 1u) ? (uint64_t)kM0 : 0ull);   // M0 * n
    const uint4 b = philox_pp(Pn, U.ctr3 + 1u, W.pp, U.k0, U.k1);
    if (ny) {
      const double L = -log_unit64(u01_64(b.x));
      if (qy <= U.dt * L) { hy = true; fy = qy / (U.dt * L); }
    }
    if (nz) {
      const double L = -log_unit64(u01_64(b.y));
      if (qz <= U.dt * L) { hz = true; fz = qz / (U.dt * L); }
    }
  }
  if (hy || hz) {
    if (cy) fy = d0y / (d0y - d1y);
    if (cz) fz = d0z / (d0z - d1z);
    if (hy && (!hz || fy <= fz)) {
      X.f = fy;
      X.wall = upy ? 1 : 3;
      double t = W.z + fy * (zn - W.z);
      t = t < U.zlo ? U.zlo : t;
      X.t = t > U.zhi ? U.zhi : t;
    } else {
      X.f = fz;
      X.wall = upz ? 2 : 0;
      double t = W.y + fz * (yn - W.y);
      t = t < U.ylo ? U.ylo : t;
      X.t = t > U.yhi ? U.yhi : t;
    }
    return true;
  }
  return false;
}

// One FP64 step.  Returns true when the step reaches the outer boundary.
template <int SIG>
__device__ __forceinline__ bool step64(const DevReq &Q, const U64<SIG> &U, W64 &W, double n0, double n1,
                                       ExitInfo<double> &X) {
  const double yn = W.y + U.s * n0;
  const double zn = W.z + U.s * n1;
  // Screen: the distance d1 of the proposal to the wall nearer the current
  // point is at least e1, its distance to its own nearer wall, so when
  // 2 d0 e1 > max(thr, 0) on both axes the proposal crossed no wall and no
  // bridge uniform is needed (rounding is monotone): the step is an ordinary
  // one, as the exact logic below would find.
  const double e1y = fmin(yn - U.ylo, U.yhi - yn), e1z = fmin(zn - U.zlo, U.zhi - zn);
  if (!((2.0 * W.dy) * e1y > U.thr0 && (2.0 * W.dz) * e1z > U.thr0) && exit64<SIG>(U, W, yn, zn, X))
    return true;
  const double c = U.reg.eval(Q, yn, zn);
  W.S = W.S + c;
  W.cc = c;
  W.y = yn;
  W.z = zn;
  W.dy = e1y;
  W.dz = e1z;
  return false;
}

__device__ __forceinline__ PathRec finish64(const DevReq &Q, const W64 &W, const ExitInfo<double> &X) {
  const double S = W.S + W.cc * X.f;
  PathRec r;
  const double2 w = finish_weight_outline(Q, X.wall, X.t, S);
  r.w_re = w.x;
  r.w_im = w.y;
  r.tau = ((double)W.n + X.f) * Q.dt;
  r.steps = W.n + 1u;
  r.wall = X.wall;
  return r;
}

// Two steps (one Philox call).  Returns 0 running, 1 exited, 2 step cap.
template <int SIG>
__device__ __forceinline__ int iterate64(const DevReq &Q, const U64<SIG> &U, W64 &W, ExitInfo<double> &X) {
  const uint4 w = philox_pp(W.P, U.ctr3, W.pp, U.k0, U.k1);
  double a0, a1, b0, b1;
  normals64(w.x, w.y, a0, a1);
  normals64(w.z, w.w, b0, b1);
  if (step64<SIG>(Q, U, W, a0, a1, X)) return 1;
  W.n += 1u;
  if (W.n >= U.max_steps) return 2;
  if (step64<SIG>(Q, U, W, b0, b1, X)) return 1;
  W.n += 1u;
  W.P += (uint64_t)kM0;
  return W.n >= U.max_steps ? 2 : 0;
}

// ===========================================================================
// FP32-mixed walk: coordinates (a, b) relative to the domain centre, walls
// at +-h.  The distance of the current point to its nearer wall, d0 = h - |a|,
// is carried from step to step.  A proposal can only reach a wall, or need a
// bridge uniform, if 2 d0 d1 <= 16.7 dt on some axis, where d1 is the distance
// of the proposal to the wall nearer to the current point; d1' = h - |a'|
// (distance to the wall nearer to the proposal) satisfies d1' <= d1, so the
// screen min(d0y d1y', d0z d1z') <= 8.35 dt never misses one.
//
// A pair of steps uses one Philox call, and one iteration of the persistent
// loop walks two pairs.  Every step updates the walker unconditionally; an
// exit is recorded in the exit info, which later steps of the iteration leave
// alone, and the walker state after an exit (or a step cap) is discarded.
// This keeps every state update in place (no per-lane merges).
// ===========================================================================
struct W32 {
  float a, b;       // y - ymid, z - zmid
  float d0y, d0z;   // h - |a|, h - |b|
  uint32_t n0, n1;  // counted signatures: full steps below the air / those in primitive 1
  uint64_t sfx;     // generic signature: phase of the full steps, units of 2^-phase_shift
  uint32_t cinc;    // generic signature: increment of the current point's region
  uint32_t n, path, node;
  uint64_t rec;
  uint64_t P;
  PhiloxPath pp;
};

// Exit of an FP32 walker: everything its record needs.
struct X32 {
  float f, t;       // fraction of the last step; tangential coordinate (centred)
  double S;         // phase at the exit point
  uint32_t n;       // index of the exit step
  int wall;         // 0 top, 1 right, 2 bottom, 3 left
};

template <int SIG> struct U32 {
  float hy, hz, thr, scr, scr_root;
  uint32_t k0, k1, ctr3, max_steps, cap2, cap2b;
  bool cap_odd;
  Reg32<SIG> reg;
  __device__ __forceinline__ void load(const DevReq &Q) {
    hy = Q.fhy; hz = Q.fhz; thr = Q.fthr; scr = Q.fscr; scr_root = Q.fscr_root;
    k0 = Q.key0; k1 = Q.key1; ctr3 = Q.ctr3; max_steps = Q.max_steps;
    cap2 = Q.cap2;
    cap2b = Q.cap2b;
    cap_odd = Q.cap_odd != 0u;
    reg.load(Q);
  }
};

// 1 + (w >> 9) 2^-23 in [1, 2): the word's top 23 bits under the exponent of 1.
__device__ __forceinline__ float one_frac32(uint32_t w) {
  return __builtin_bit_cast(float, __builtin_amdgcn_alignbit(0x7Fu, w, 9u));
}
// (2 (w >> 9) + 1) 2^-24: exact in FP32 (the subtraction is exact), in (0, 1).
__device__ __forceinline__ float u01_32(uint32_t w) { return one_frac32(w) - 0x1.fffffep-1f; }

// dt (-ln U) in the FP32 walk's squared length unit K^2 = 2 ln 2 dt:
// -log2(U) / 2.
__device__ __forceinline__ float bridge_len32(uint32_t w) { return -0.5f * __builtin_amdgcn_logf(u01_32(w)); }

// Box-Muller and the Euler-Maruyama proposal in one: with the hardware log2,
// sqrt(-2 ln u) sqrt(dt) = K sqrt(-log2 u), K = sqrt(dt) sqrt(2 ln 2), and
// positions are in units of K; the angle is in revolutions (v_sin/v_cos_f32),
// and 1 + k 2^-23 is the same angle as k 2^-23.
__device__ __forceinline__ void propose32(float a, float b, uint32_t wa, uint32_t wb, float &an, float &bn) {
  const float rk = __builtin_amdgcn_sqrtf(-__builtin_amdgcn_logf(u01_32(wa)));
  const float ang = one_frac32(wb);
  an = __builtin_fmaf(__builtin_amdgcn_cosf(ang), rk, a);
  bn = __builtin_fmaf(__builtin_amdgcn_sinf(ang), rk, b);
}

template <int SIG>
__device__ __forceinline__ void start32(const DevReq &Q, const U32<SIG> &U, W32 &W, uint32_t node, uint32_t path,
                                        uint64_t rec) {
  const double2 p = *reinterpret_cast<const double2 *>(Q.nodes + 2 * (size_t)node);
  W.a = (float)((p.x - Q.ymid) * Q.kinv);
  W.b = (float)((p.y - Q.zmid) * Q.kinv);
  W.d0y = U.hy - fabsf(W.a);
  W.d0z = U.hz - fabsf(W.b);
  W.n0 = 0;
  W.n1 = 0;
  W.sfx = 0;
  if constexpr (Reg32<SIG>::kGeneric) W.cinc = U.reg.inc32(Q, W.a, W.b);
  W.n = 0;
  W.path = path;
  W.node = node;
  W.rec = rec;
  W.P = 0;
  W.pp = philox_path(path, node, U.k0);
}

// Exact exit logic for a lane the screen flagged (step index nstep).
template <int SIG>
__device__ __forceinline__ bool exit32(const DevReq &Q, const U32<SIG> &U, const W32 &W, float an, float bn,
                                       uint32_t nstep, X32 &X) {
  const bool upy = W.a > 0.f;   // a tie (a = 0) goes to the lower wall
  const bool upz = W.b > 0.f;
  const float d0y = W.d0y, d0z = W.d0z;
  const float d1y = upy ? (U.hy - an) : (U.hy + an);
  const float d1z = upz ? (U.hz - bn) : (U.hz + bn);
  const bool cy = d1y <= 0.f, cz = d1z <= 0.f;
  const float qy = (2.f * d0y) * d1y, qz = (2.f * d0z) * d1z;
  bool hy = cy, hz = cz;
  float fy = 0.f, fz = 0.f;
  const bool ny = !cy && (qy <= U.thr);
  const bool nz = !cz && (qz <= U.thr);
  if (ny || nz) {
    const uint64_t Pn = (W.P << 1) + ((nstep & 1u) ? (uint64_t)kM0 : 0ull);
    const uint4 u = philox_pp(Pn, U.ctr3 + 1u, W.pp, U.k0, U.k1);
    if (ny) {
      const float L = bridge_len32(u.x);
      if (qy <= L) { hy = true; fy = qy * __builtin_amdgcn_rcpf(L); }
    }
    if (nz) {
      const float L = bridge_len32(u.y);
      if (qz <= L) { hz = true; fz = qz * __builtin_amdgcn_rcpf(L); }
    }
  }
  if (!(hy || hz)) return false;
  // fractions from the hardware reciprocal (1 ulp), kept in [0, 1]
  if (cy) fy = d0y * __builtin_amdgcn_rcpf(d0y - d1y);
  if (cz) fz = d0z * __builtin_amdgcn_rcpf(d0z - d1z);
  float f;
  if (hy && (!hz || fy <= fz)) {
    f = fminf(fy, 1.f);
    X.wall = upy ? 1 : 3;
    X.t = fminf(fmaxf(__builtin_fmaf(f, bn - W.b, W.b), -U.hz), U.hz);
  } else {
    f = fminf(fz, 1.f);
    X.wall = upz ? 2 : 0;
    X.t = fminf(fmaxf(__builtin_fmaf(f, an - W.a, W.a), -U.hy), U.hy);
  }
  X.f = f;
  X.n = nstep;
  // phase of the nstep full steps, plus the partial step charged to the
  // region of the last inside point
  if constexpr (Reg32<SIG>::kCounted) {
    X.S = U.reg.phase(Q, W.n0, W.n1, nstep) + U.reg.rate(Q, U.reg.index(Q, W.a, W.b)) * (double)f;
  } else {
    X.S = __builtin_ldexp((double)W.sfx + (double)W.cinc * (double)f, -Q.phase_shift);
  }
  return true;
}

// A full step to (an, bn): the walker moves there and the step's phase goes
// to the region of that point (right-point rule): a step count per region,
// or (generic signature) the region's fixed-point increment added to the
// 64-bit sum.
template <int SIG>
__device__ __forceinline__ void advance32(const DevReq &Q, const U32<SIG> &U, W32 &W, float an, float bn, float e1y,
                                          float e1z) {
  if constexpr (Reg32<SIG>::kCounted) {
    U.reg.count(an, bn, W.n0, W.n1);
  } else {
    const uint32_t c = U.reg.inc32(Q, an, bn);
    W.sfx += c;
    W.cinc = c;
  }
  W.a = an;
  W.b = bn;
  W.d0y = e1y;
  W.d0z = e1z;
}

template <bool kOutline>
__device__ __forceinline__ PathRec finish32(const DevReq &Q, const X32 &X) {
  const double S = X.S;
  const bool along_y = (X.wall == 0) || (X.wall == 2);
  double t = (double)X.t * Q.kscale + (along_y ? Q.ymid : Q.zmid);
  const double lo = along_y ? Q.y_lo : Q.z_lo, hi = along_y ? Q.y_hi : Q.z_hi;
  t = t < lo ? lo : (t > hi ? hi : t);
  PathRec r;
  if constexpr (kOutline) {
    const double2 w = finish_weight_outline(Q, X.wall, t, S);
    r.w_re = w.x;
    r.w_im = w.y;
  } else {
    finish_weight(Q, X.wall, t, S, r);
  }
  r.tau = ((double)X.n + (double)X.f) * Q.dt;
  r.steps = X.n + 1u;
  r.wall = X.wall;
  return r;
}

__device__ __forceinline__ int32_t fbits(float x) { return __builtin_bit_cast(int32_t, x); }

// Two steps (one Philox call).  Both proposals are made first; a step needs
// its exact exit logic only if its screen min(d0y d1y', d0z d1z') <= scr
// flags it, which needs some distance of the pair's three points at or below
// r = scr_root (every product of two distances above r exceeds scr in FP32),
// so one test of the least of the six distances clears both steps in all but
// a few percent of pairs.  The walker always advances; `stop` (the lane's
// walk ended in an earlier pair: exit, recorded in X, or step cap) skips the
// exit logic, and the state after a stop is discarded.
template <int SIG, int K>
__device__ __forceinline__ void pair32(const DevReq &Q, const U32<SIG> &U, W32 &W, X32 &X, uint32_t n0, bool &ex,
                                       bool &stop) {
  const uint4 w = philox_pp(W.P, U.ctr3, W.pp, U.k0, U.k1);
  const uint32_t n = n0 + 2u * K;   // index of the pair's first step (K: the pair within the iteration)
  float a1, b1, a2, b2;
  propose32(W.a, W.b, w.x, w.y, a1, b1);
  propose32(a1, b1, w.z, w.w, a2, b2);
  const float e1y = U.hy - fabsf(a1), e1z = U.hz - fabsf(b1);
  const float e2y = U.hy - fabsf(a2), e2z = U.hz - fabsf(b2);
  // least distance compared through the bit patterns: for r > 0, x <= r iff
  // the signed integer reading of x is <= that of r (negative x, -0 included,
  // read as negative integers), and integer minima need no NaN handling
  const int32_t m =
      min(min(min(min(min(fbits(W.d0y), fbits(W.d0z)), fbits(e1y)), fbits(e1z)), fbits(e2y)), fbits(e2z));
  // step caps (n is even here): the pair is the last one when n >= cap2, and
  // its first step is then the last allowed iff max_steps is odd
  const bool near = K == 0 ? (n0 >= U.cap2) : (n0 >= U.cap2b);
  const bool capA = near && U.cap_odd;
  const W32 W0 = W;   // the walker before the pair, for the first step's exit logic
  advance32<SIG>(Q, U, W, a1, b1, e1y, e1z);
  if (!stop && m <= fbits(U.scr_root)) {
    if (fminf(W0.d0y * e1y, W0.d0z * e1z) <= U.scr) ex = exit32<SIG>(Q, U, W0, a1, b1, n, X);
    if (!ex && !capA && fminf(e1y * e2y, e1z * e2z) <= U.scr) ex = exit32<SIG>(Q, U, W, a2, b2, n + 1u, X);
  }
  advance32<SIG>(Q, U, W, a2, b2, e2y, e2z);
  W.P += (uint64_t)kM0;
  stop = stop || ex || near;
}

// Four steps, two pairs.  Returns 0 running, 1 exited, 2 step cap.  With two
// pairs per call the walker state alternates between two register sets (a
// pair's old state is live until its exit logic, after its new state
// exists), so no copies close the loop; a lane whose walk ends in the first
// pair idles for two steps, against paths of thousands of steps.
template <int SIG>
__device__ __forceinline__ int iterate32(const DevReq &Q, const U32<SIG> &U, W32 &W, X32 &X) {
  bool ex = false, stop = false;
  const uint32_t n0 = W.n;
  pair32<SIG, 0>(Q, U, W, X, n0, ex, stop);
  pair32<SIG, 1>(Q, U, W, X, n0, ex, stop);
  W.n = n0 + 4u;
  return ex ? 1 : (stop ? 2 : 0);
}

// Precision traits for the persistent loop (kPairs: pairs of steps per
// iterate call, the unit of the slice budget).
template <int SIG> struct F64 {
  static constexpr uint32_t kPairs = 1;
  using Walker = W64;
  using Uni = U64<SIG>;
  using Exit = ExitInfo<double>;
  static __device__ __forceinline__ void start(const DevReq &Q, const Uni &U, Walker &W, uint32_t node,
                                               uint32_t path, uint64_t rec) { start64<SIG>(Q, U, W, node, path, rec); }
  static __device__ __forceinline__ int iterate(const DevReq &Q, const Uni &U, Walker &W, Exit &X) {
    return iterate64<SIG>(Q, U, W, X);
  }
  static __device__ __forceinline__ PathRec finish(const DevReq &Q, const Walker &W, const Exit &X) {
    return finish64(Q, W, X);
  }
  // Suspension at a slice boundary (n is even there) and exact resumption.
  static __device__ __forceinline__ void save(const Walker &W, SuspRec &s) {
    s.x = W.y; s.y = W.z; s.s_hi = W.S; s.s_lo = 0.0; s.rec = W.rec;
    s.n = W.n; s.path = W.path; s.node = W.node; s.pad = 0; s.pad1 = 0;
  }
  static __device__ __forceinline__ void resume(const DevReq &Q, const Uni &U, Walker &W, const SuspRec &s) {
    W.y = s.x; W.z = s.y; W.S = s.s_hi; W.rec = s.rec; W.n = s.n; W.path = s.path; W.node = s.node;
    W.P = (uint64_t)kM0 * (uint64_t)(W.n >> 1);
    W.pp = philox_path(W.path, W.node, U.k0);
    W.cc = U.reg.eval(Q, W.y, W.z);
    W.dy = fmin(W.y - U.ylo, U.yhi - W.y);
    W.dz = fmin(W.z - U.zlo, U.zhi - W.z);
  }
};
template <int SIG> struct F32 {
  static constexpr uint32_t kPairs = 2;
  using Walker = W32;
  using Uni = U32<SIG>;
  using Exit = X32;
  static __device__ __forceinline__ void start(const DevReq &Q, const Uni &U, Walker &W, uint32_t node,
                                               uint32_t path, uint64_t rec) { start32<SIG>(Q, U, W, node, path, rec); }
  static __device__ __forceinline__ int iterate(const DevReq &Q, const Uni &U, Walker &W, Exit &X) {
    return iterate32<SIG>(Q, U, W, X);
  }
  static __device__ __forceinline__ PathRec finish(const DevReq &Q, const Walker &, const Exit &X) {
    return finish32<Reg32<SIG>::kGeneric>(Q, X);
  }
  // counts and FP32 values all widen to doubles exactly; the generic
  // signature's 64-bit phase sum and increment go to the integer fields
  static __device__ __forceinline__ void save(const Walker &W, SuspRec &s) {
    s.x = (double)W.a; s.y = (double)W.b;
    s.s_hi = Reg32<SIG>::kCounted ? (double)W.n0 : 0.0;
    s.s_lo = Reg32<SIG>::kCounted ? (double)W.n1 : 0.0;
    s.rec = W.rec; s.n = W.n; s.path = W.path; s.node = W.node;
    s.pad = Reg32<SIG>::kCounted ? 0u : W.cinc;
    s.pad1 = Reg32<SIG>::kCounted ? 0ull : W.sfx;
  }
  static __device__ __forceinline__ void resume(const DevReq &Q, const Uni &U, Walker &W, const SuspRec &s) {
    W.a = (float)s.x; W.b = (float)s.y;
    if constexpr (Reg32<SIG>::kCounted) {
      W.n0 = (uint32_t)s.s_hi; W.n1 = (uint32_t)s.s_lo;
    } else {
      W.sfx = s.pad1; W.cinc = s.pad;
    }
    W.rec = s.rec; W.n = s.n; W.path = s.path; W.node = s.node;
    W.d0y = U.hy - fabsf(W.a);
    W.d0z = U.hz - fabsf(W.b);
    W.P = (uint64_t)kM0 * (uint64_t)(W.n >> 1);
    W.pp = philox_path(W.path, W.node, U.k0);
  }
};

// ---------------------------------------------------------------------------
// Plain FP64 walker: one thread walks one path to its end.
// ---------------------------------------------------------------------------
template <int SIG>
__device__ __forceinline__ void plain_body(const DevReq &Q, uint32_t node, uint32_t p0, uint32_t count,
                                           uint64_t rec0) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= count) return;
  U64<SIG> U;
  U.load(Q);
  W64 W;
  start64<SIG>(Q, U, W, node, p0 + tid, rec0 + tid);
  ExitInfo<double> X;
  int st = W.n >= U.max_steps ? 2 : 0;
  while (st == 0) st = iterate64<SIG>(Q, U, W, X);
  Q.recs[W.rec] = st == 1 ? finish64(Q, W, X) : unfinished_rec(U.max_steps);
}

__global__ void __launch_bounds__(256) walk_plain(const DevReq *__restrict__ reqs, uint32_t node, uint32_t p0,
                                                  uint32_t count, uint64_t rec0) {
  const DevReq &Q = reqs[0];
  switch (Q.sig) {
    case kSigNone: plain_body<kSigNone>(Q, node, p0, count, rec0); break;
    case kSigZ: plain_body<kSigZ>(Q, node, p0, count, rec0); break;
    case kSigZY: plain_body<kSigZY>(Q, node, p0, count, rec0); break;
    case kSigZBox: plain_body<kSigZBox>(Q, node, p0, count, rec0); break;
    case kSigZTri: plain_body<kSigZTri>(Q, node, p0, count, rec0); break;
    default: plain_body<kSigGeneric>(Q, node, p0, count, rec0); break;
  }
}

// ---------------------------------------------------------------------------
// Persistent walker.
// ---------------------------------------------------------------------------
// Work a request still has: unclaimed tiles, tile remainders and suspended
// walkers left by the previous slice (a rough count in tiles).
__device__ __forceinline__ uint32_t work_left(const DevReq &Q) {
  const uint32_t taken = uni(__hip_atomic_load(Q.tile_counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  uint32_t left = taken < Q.n_tiles ? Q.n_tiles - taken : 0u;
  if (Q.slice_ctl) {
    const uint32_t pc = uni(__hip_atomic_load(Q.slice_ctl + kPoolCursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const uint32_t ec = uni(__hip_atomic_load(Q.slice_ctl + kExtraCursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    left += ec < Q.extra_in_n ? Q.extra_in_n - ec : 0u;
    left += pc < Q.pool_in_n ? (Q.pool_in_n - pc + 63u) / 64u : 0u;
  }
  return left;
}

__device__ __forceinline__ uint32_t pick_request(const DevReq *__restrict__ reqs, uint32_t n_req) {
  // the request with the most work left (ties: lowest index)
  uint32_t best = kNoRequest, best_left = 0;
  for (uint32_t r = 0; r < n_req; ++r) {
    const uint32_t left = work_left(reqs[r]);
    if (left > best_left) { best_left = left; best = r; }
  }
  return best;
}

// Walk request Q with this wave until its work runs out (returns false) or
// the wave's slice budget is spent (returns true: in-flight walkers and the
// tile remainder were suspended for the next slice).  budget == 0: no limit.
template <class T>
__device__ __forceinline__ bool run_request(const DevReq &Q, uint32_t budget, uint32_t refill_mask, uint32_t &iters) {
  const uint32_t lane = __lane_id();
  typename T::Uni U;
  U.load(Q);
  const uint32_t n_tiles = Q.n_tiles;
  uint32_t *ctl = Q.slice_ctl;
  typename T::Walker W;
  bool active = false;

  // wave-uniform cursors
  uint32_t t_node = 0, t_p0 = 0, t_next = 0, t_end = 0;
  uint64_t t_rec0 = 0;
  bool pool_done = (ctl == nullptr) || (Q.pool_in_n == 0u);
  bool extra_done = (ctl == nullptr) || (Q.extra_in_n == 0u);
  bool exhausted = false;
  bool suspended = false;
  uint32_t finished = 0;   // paths this lane completed

  for (;;) {
    uint64_t freemask = __builtin_amdgcn_ballot_w64(!active);
    // refill every (refill_mask + 1) pairs of steps (`iters` counts pairs), and
    // whenever every lane is idle
    const bool refill = ((iters & refill_mask) == 0u) || (freemask == ~0ull);
    if (!refill) freemask = 0ull;
    // (with every lane busy, or between refills, nothing below changes `active`)
    if (freemask != 0ull) {
      // resume walkers suspended by the previous slice first
      if (!pool_done) {
        const uint32_t nfree = (uint32_t)__popcll(freemask);
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(freemask >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)freemask, 0u));
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(ctl + kPoolCursor, nfree);
        base = uni(base);
        const uint32_t avail = base < Q.pool_in_n ? min(nfree, Q.pool_in_n - base) : 0u;
        if (avail < nfree) pool_done = true;
        if (!active && rank < avail) {
          T::resume(Q, U, W, Q.pool_in[base + rank]);
          active = true;
        }
        freemask = __builtin_amdgcn_ballot_w64(!active);
      }
      // then refill free lanes in rank order from the wave's tile, claiming
      // tile remainders of the previous slice before new tiles
      if (freemask != 0ull && !exhausted) {
        const uint32_t nfree = (uint32_t)__popcll(freemask);
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(freemask >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)freemask, 0u));
        uint32_t given = 0;
        while (given < nfree) {
          if (t_next == t_end) {
            const DevTile *src = nullptr;
            if (!extra_done) {
              uint32_t e = 0;
              if (lane == 0) e = atomicAdd(ctl + kExtraCursor, 1u);
              e = uni(e);
              if (e < Q.extra_in_n) src = Q.extra_in + e;
              else extra_done = true;
            }
            if (src == nullptr) {
              // a request whose tiles are all claimed is left alone: the
              // counter moves past n_tiles only in a race between waves
              // that both saw a tile left (at most one step per wave)
              uint32_t t = n_tiles;
              if (lane == 0) {
                t = __hip_atomic_load(Q.tile_counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (t < n_tiles) t = atomicAdd(Q.tile_counter, 1u);
              }
              t = uni(t);
              if (t >= n_tiles) { exhausted = true; break; }
              src = Q.tiles + t;
            }
            const DevTile Tl = *src;
            t_node = uni(Tl.node);
            t_p0 = uni(Tl.p0);
            t_next = t_p0;
            t_end = t_p0 + uni(Tl.count);
            t_rec0 = ((uint64_t)uni((uint32_t)(Tl.rec0 >> 32)) << 32) | uni((uint32_t)Tl.rec0);
          }
          const uint32_t take = min(t_end - t_next, nfree - given);
          if (!active && rank >= given && rank < given + take) {
            const uint32_t p = t_next + (rank - given);
            T::start(Q, U, W, t_node, p, t_rec0 + (p - t_p0));
            active = true;
          }
          t_next += take;
          given += take;
        }
      }
      // every lane idle after a refill: this wave can get no more work here
      if (__builtin_amdgcn_ballot_w64(!active) == ~0ull) break;
    }

    if (active) {
      typename T::Exit X;
      const int st = T::iterate(Q, U, W, X);
      if (st != 0) {
        Q.recs[W.rec] = st == 1 ? T::finish(Q, W, X) : unfinished_rec(U.max_steps);
        active = false;
        finished += 1u;
      }
    }
    iters += T::kPairs;
    if (budget != 0u && iters >= budget) {
      // suspend: in-flight walkers to pool_out, the tile remainder to extra_out
      const uint64_t am = __builtin_amdgcn_ballot_w64(active);
      const uint32_t cnt = (uint32_t)__popcll(am);
      if (cnt) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(ctl + kPoolOut, cnt);
        base = uni(base);
        const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(am >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)am, 0u));
        // the host sizes pool_out for every lane of the launch; a count past
        // the capacity is reported to it (the walker is not written)
        if (active && base + r < Q.pool_cap) T::save(W, Q.pool_out[base + r]);
      }
      if (t_next != t_end) {   // (modular: a tile may end at path 2^32)
        uint32_t e = 0;
        if (lane == 0) e = atomicAdd(ctl + kExtraOut, 1u);
        e = uni(e);
        if (lane == 0 && e < Q.extra_cap) {
          DevTile Tl;
          Tl.node = t_node;
          Tl.p0 = t_next;
          Tl.count = t_end - t_next;
          Tl.pad = 0;
          Tl.rec0 = t_rec0 + (t_next - t_p0);
          Tl.pad1 = 0;
          Q.extra_out[e] = Tl;
        }
      }
      suspended = true;
      break;
    }
  }
  if (finished) atomicAdd(Q.done_counter, (unsigned long long)finished);
  return suspended;
}

// A launch mixing signatures runs each request's walker loop inlined in one
// dispatching kernel, except the generic signature's, whose registers (the
// sigma grid's parameters, the primitive list) would otherwise push the
// others' loop-invariant values into spill slots: it is called out of line.
template <class T>
__device__ __noinline__ bool run_request_outline(const DevReq &Q, uint32_t budget, uint32_t refill_mask, uint32_t &iters) {
  return run_request<T>(Q, budget, refill_mask, iters);
}

template <template <int> class T>
__device__ __forceinline__ bool run_dispatch(const DevReq &Q, uint32_t budget, uint32_t refill_mask, uint32_t &iters) {
  switch (uni((uint32_t)Q.sig)) {
    case kSigNone: return run_request<T<kSigNone>>(Q, budget, refill_mask, iters);
    case kSigZ: return run_request<T<kSigZ>>(Q, budget, refill_mask, iters);
    case kSigZY: return run_request<T<kSigZY>>(Q, budget, refill_mask, iters);
    case kSigZBox: return run_request<T<kSigZBox>>(Q, budget, refill_mask, iters);
    case kSigZTri: return run_request<T<kSigZTri>>(Q, budget, refill_mask, iters);
    default: return run_request_outline<T<kSigGeneric>>(Q, budget, refill_mask, iters);
  }
}

// SIG >= 0: every request of the launch has model signature SIG (the walker
// is compiled for it alone, which keeps the register allocation of the other
// signatures out of the loop); SIG < 0: requests of any signature.
template <template <int> class T, int SIG>
__device__ __forceinline__ bool run_sig(const DevReq &Q, uint32_t budget, uint32_t refill_mask, uint32_t &iters) {
  if constexpr (SIG < 0) return run_dispatch<T>(Q, budget, refill_mask, iters);
  else return run_request<T<SIG>>(Q, budget, refill_mask, iters);
}

template <template <int> class T, int SIG>
__device__ __forceinline__ void persist_body(const DevReq *__restrict__ reqs, uint32_t n_req,
                                             const uint32_t *__restrict__ wave_start, uint32_t budget,
                                             uint32_t refill_mask) {
  const uint32_t wid = uni((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  // initial request: waves are shared out in proportion to each request's work
  uint32_t r = kNoRequest;
  for (uint32_t i = 0; i < n_req; ++i)
    if (wid >= wave_start[i] && wid < wave_start[i + 1]) r = i;
  r = uni(r);
  if (r == kNoRequest) r = pick_request(reqs, n_req);
  // Each visit either claims work or finds the request's work gone, after
  // which pick_request never returns it again (claim cursors only grow): the
  // loop ends once all work is claimed, or at the slice budget.
  uint32_t iters = 0;
  while (r != kNoRequest) {
    if (run_sig<T, SIG>(reqs[r], budget, refill_mask, iters)) break;
    r = pick_request(reqs, n_req);
  }
}

template <int SIG>
__global__ void __launch_bounds__(256) walk_persist_f64(const DevReq *__restrict__ reqs, uint32_t n_req,
                                                        const uint32_t *__restrict__ wave_start, uint32_t budget,
                                                        uint32_t refill_mask) {
  persist_body<F64, SIG>(reqs, n_req, wave_start, budget, refill_mask);
}

template <int SIG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) walk_persist_f32(const DevReq *__restrict__ reqs, uint32_t n_req,
                                                        const uint32_t *__restrict__ wave_start, uint32_t budget,
                                                        uint32_t refill_mask) {
  persist_body<F32, SIG>(reqs, n_req, wave_start, budget, refill_mask);
}

// The generic signature with the sigma grid staged in LDS: every request of
// the launch shares one grid (the same model, time step and frequency), whose
// class table and class bytes each block copies into LDS once.  Blocks of 768
// threads, two per CU (the LDS form of a 256 x 224 grid is about 60 KB), so
// a CU holds 24 waves as the 256-thread walkers do.
constexpr uint32_t kLdsThreads = 768;
__global__ void __launch_bounds__(kLdsThreads) __attribute__((amdgpu_waves_per_eu(6, 8))) walk_persist_f32_lds(const DevReq *__restrict__ reqs, uint32_t n_req,
                                                                     const uint32_t *__restrict__ wave_start,
                                                                     uint32_t budget, uint32_t refill_mask) {
  const uint4 *src = reinterpret_cast<const uint4 *>(reqs[0].lds_src);
  const uint32_t n16 = reqs[0].lds_bytes / 16u;
  for (uint32_t i = threadIdx.x; i < n16; i += blockDim.x) reinterpret_cast<uint4 *>(g_lds)[i] = src[i];
  __syncthreads();
  persist_body<F32, kSigGenericLds>(reqs, n_req, wave_start, budget, refill_mask);
}

using PersistKernel = void (*)(const DevReq *, uint32_t, const uint32_t *, uint32_t, uint32_t);

template <int SIG> struct K64 { static constexpr PersistKernel fn = walk_persist_f64<SIG>; };
template <int SIG> struct K32 { static constexpr PersistKernel fn = walk_persist_f32<SIG>; };

template <template <int> class K>
static PersistKernel pick_kernel(int sig) {
  switch (sig) {
    case kSigNone: return K<kSigNone>::fn;
    case kSigZ: return K<kSigZ>::fn;
    case kSigZY: return K<kSigZY>::fn;
    case kSigZBox: return K<kSigZBox>::fn;
    case kSigZTri: return K<kSigZTri>::fn;
    case kSigGeneric: return K<kSigGeneric>::fn;
    default: return K<-1>::fn;
  }
}

static PersistKernel persist_kernel(int precision, int sig) {
  if (precision != 0 && sig == kSigGenericLds) return walk_persist_f32_lds;
  return precision == 0 ? pick_kernel<K64>(sig) : pick_kernel<K32>(sig);
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

// Statistics of one node from its records, two passes in a fixed order;
// REC(i) gives path i's (valid, w_re, w_im, tau, steps).
struct RecView {
  bool done;
  double w_re, w_im, tau;
  uint32_t steps;
};

template <class REC>
__device__ __forceinline__ void reduce_body(uint64_t count, const REC &rec, NodeOut *out) {
  __shared__ double lds[kRedThreads / 64][4];
  __shared__ unsigned long long ldsu[kRedThreads / 64][3];
  const int tid = threadIdx.x;
  double s[4] = {0.0, 0.0, 0.0, 0.0};  // sum re, sum im, sum tau, (unused)
  unsigned long long cnt[3] = {0ull, 0ull, 0ull};  // done, unfinished, steps
  for (uint64_t i = tid; i < count; i += kRedThreads) {
    const RecView r = rec(i);
    cnt[2] += r.steps;
    if (!r.done) { cnt[1] += 1ull; continue; }
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
    const RecView r = rec(i);
    if (!r.done) continue;
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
    *out = o;
  }
}

__global__ void __launch_bounds__(kRedThreads) reduce_nodes(const NodeJob *__restrict__ jobs) {
  const NodeJob J = jobs[blockIdx.x];
  auto rec = [&](uint64_t i) {
    const PathRec r = i < J.count0 ? J.recs0[i] : J.recs1[i - J.count0];
    return RecView{r.wall >= 0, r.w_re, r.w_im, r.tau, r.steps};
  };
  reduce_body(J.count0 + J.count1, rec, J.out);
}

// Multi-frequency results: path i's weight at this job's frequency is
// g_f(exit point) exp(-i scale S), from the phase record of the one walk.
__global__ void __launch_bounds__(kRedThreads) reduce_fanout(const FanJob *__restrict__ jobs, int M, double y_lo,
                                                              double y_hi, double z_lo, double z_hi) {
  const FanJob J = jobs[blockIdx.x];
  auto rec = [&](uint64_t i) {
    const PathRec r = J.recs[i];
    RecView v{r.wall >= 0, 0.0, 0.0, r.tau, r.steps};
    if (v.done) weight_tab(J.g, M, y_lo, y_hi, z_lo, z_hi, r.wall, r.w_im, J.scale * r.w_re, v.w_re, v.w_im);
    return v;
  };
  reduce_body(J.count, rec, J.out);
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

// lds_bytes: the dynamic LDS of the kSigGenericLds walker (the grid's LDS
// form), 0 for every other build.
hipError_t launch_walk_persist(int precision, int sig, const DevReq *reqs_dev, uint32_t n_req,
                               const uint32_t *wave_start_dev, uint32_t budget, uint32_t refill_mask, uint32_t blocks,
                               uint32_t threads, uint32_t lds_bytes, hipStream_t st) {
  hipLaunchKernelGGL(persist_kernel(precision, sig), dim3(blocks), dim3(threads), lds_bytes, st, reqs_dev, n_req,
                     wave_start_dev, budget, refill_mask);
  return hipGetLastError();
}

int persist_blocks_per_cu(int precision, int sig, uint32_t threads, uint32_t lds_bytes) {
  int nb = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, persist_kernel(precision, sig), (int)threads,
                                                                    lds_bytes);
  return e == hipSuccess ? nb : 0;
}

uint32_t lds_walker_threads() { return kLdsThreads; }

hipError_t launch_reduce_fanout(const FanJob *jobs_dev, uint32_t n_jobs, int M, double y_lo, double y_hi, double z_lo,
                                double z_hi, hipStream_t st) {
  if (n_jobs == 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_fanout, dim3(n_jobs), dim3(kRedThreads), 0, st, jobs_dev, M, y_lo, y_hi, z_lo, z_hi);
  return hipGetLastError();
}

hipError_t launch_reduce(const NodeJob *jobs_dev, uint32_t n_jobs, hipStream_t st) {
  if (n_jobs == 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_nodes, dim3(n_jobs), dim3(kRedThreads), 0, st, jobs_dev);
  return hipGetLastError();
}

hipError_t launch_reset(uint32_t *tile_counters, unsigned long long *done, uint32_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(reset_counters, dim3((n + 255u) / 256u), dim3(256), 0, st, tile_counters, done, n);
  return hipGetLastError();
}

}  // namespace sdd
