// Device-side data layout shared by the kernels and the host runtime.
//
// Everything a wave needs for one request lives in a DevReq that the wave
// reads with scalar loads (the request index is wave-uniform), so the model,
// the step size, the phase increments and the Philox key sit in SGPRs and the
// 64 lanes hold only their walkers' state in VGPRs.
#pragma once
#include <stdint.h>

namespace sdd {

constexpr int kMaxPrims = 16;                 // conductivity primitives per model
constexpr int kMaxRegions = kMaxPrims + 1;    // + background
constexpr int kPfStride = 12;                 // FP32 parameters per primitive (DevReq::pf)
constexpr uint32_t kNoRequest = 0xFFFFFFFFu;

enum PrimKind : int32_t { kHalfZ = 0, kHalfY = 1, kBox = 2, kTriangle = 3 };

// Model signatures with a specialised, branch-free region lookup; any other
// model uses the generic lookup: the sigma grid (in global memory, or staged
// in LDS when every request of a launch shares one grid: kSigGenericLds) or
// the loop over its primitives.
enum ModelSig : int32_t {
  kSigNone = 0, kSigZ = 1, kSigZY = 2, kSigZBox = 3, kSigZTri = 4, kSigGeneric = 5, kSigGenericLds = 6
};

// Resident conductivity model (workspace copy made by sdd_model_create).  The
// walkers read the primitives from each request's DevReq (converted there to
// the request's centred FP32 coordinates); this copy is the model's device
// footprint, counted against the workspace while the model is resident.
struct DevModel {
  int32_t nprims;
  int32_t pad0[3];
  int32_t kind[kMaxPrims];
  double pd[kMaxPrims][6];    // FP64 geometry
  float pf[kMaxPrims][8];     // FP32 geometry (FP32-mixed walks), padded to 8
  double sigma[kMaxRegions];  // per region, background last
  double y_lo, y_hi, z_lo, z_hi, length_unit_m, pad1[3];
};

// A work unit claimed by a wave: `count` consecutive paths of one node.
struct DevTile {
  uint32_t node;
  uint32_t p0;        // first path index
  uint32_t count;
  uint32_t pad;
  uint64_t rec0;      // record slot of path p0 (request-relative)
  uint64_t pad1;
};

// A walker suspended at the end of a time slice (served mode), 64 bytes.
// Positions and phase are stored exactly (FP32 values widen losslessly);
// everything else a walker holds is recomputed from these on resume.
struct SuspRec {
  double x, y;         // FP64 walk: (y, z); FP32 walk: centred (a, b)
  double s_hi, s_lo;   // phase
  uint64_t rec;        // record slot
  uint32_t n, path, node, pad;
  uint64_t pad1;
};

// Per-request slice control words: claim cursors and append counts.
enum SliceCtl : int { kPoolCursor = 0, kPoolOut = 1, kExtraCursor = 2, kExtraOut = 3 };

// Per-path record, 32 bytes.
struct PathRec {
  double w_re, w_im;
  double tau;          // (n + f) dt, or -1 when unfinished
  uint32_t steps;      // proposals drawn
  int32_t wall;        // 0 top, 1 right, 2 bottom, 3 left, -1 unfinished
};

// Per-node reduction output, 96 bytes.
struct NodeOut {
  double mean_re, mean_im, var_re, var_im, cov, se_re, se_im, se, mean_exit_time;
  uint64_t paths_done, steps, unfinished;
};

// One node's records for the reduction kernel: up to two segments (the
// pilot and the extension of a target-SE request), reduced in that order.
struct NodeJob {
  const PathRec *recs0;
  uint64_t count0;
  const PathRec *recs1;
  uint64_t count1;
  NodeOut *out;
  uint64_t pad;
};

// One (node, frequency) result of a multi-frequency solve: the node's phase
// records weighted with the frequency's boundary tables and phase scale.
struct FanJob {
  const PathRec *recs;
  uint64_t count;
  const double *g;     // 4 x (M + 1) x (re, im) at this frequency
  double scale;        // frequency / the walk's frequency
  NodeOut *out;
  uint64_t pad;
};

// One cell of the sigma grid of the FP32 walk's generic signature (32 B):
// the phase increment of a full step ending at a point (a, b) of the cell
// (fixed point: units of 2^-phase_shift) is inc_ge if the edge function
//   e = fma(A, a, fma(B, b, C))   (FP32)
// is >= 0, else inc_lt.  Lines are the primitive loop's own: a box side or
// half-plane a < y0 reads A = 1, B = 0, C = -y0 (e = a - y0 rounded once, so
// its sign is the compare's), a triangle edge its oriented (A, B, C) from
// DevReq::pf.  A line's increments are swapped where the loop's test is
// e < 0, so that every test reads "e >= 0" with the two increments in the
// right order.  A pure
// cell has A = B = C = 0 (e = +0) and equal increments.  A cell whose
// primitives test two lines has bit 30 of inc_ge set (kCellTwo; increments
// are below 2^30): its increment is inc_ge or inc_lt when e2 < 0 and the
// extension entry's inc_ge (e >= 0) or inc_lt (e < 0) when e2 >= 0, e2 the
// extension entry's line; xi is the extension's index.  A cell with more
// lines has bit 31 set (kCellLoop): its points take the primitive loop.  The
// LDS form of a grid stores one class byte per cell, then each distinct cell
// once (a class table of at most 255 SigmaCells, then the extension
// entries).
constexpr uint32_t kCellLoop = 0x80000000u;
constexpr uint32_t kCellTwo = 0x40000000u;
constexpr uint32_t kCellFlags = kCellLoop | kCellTwo;
constexpr uint32_t kMaxLdsClasses = 255;
struct SigmaCell {
  uint32_t inc_ge, inc_lt;
  float A, B, C;
  uint32_t xi;
  uint32_t pad[2];
};

// Per-request device descriptor.
struct DevReq {
  // FP64 walk (absolute coordinates, the same arithmetic as a plain FP64 reference)
  double y_lo, y_hi, z_lo, z_hi;
  double s;            // sqrt(dt)
  double dt;
  double thr;          // bridge pre-filter: draw U only if 2 d0 d1 <= thr
  double ymid, zmid;   // centre of the domain (origin of the FP32 walk)
  double kscale;       // K = sqrt(dt) sqrt(2 ln 2), the FP32 walk's length unit
  double kinv;         // 1 / K
  double c[kMaxRegions + 1];   // phase per full step: alpha_r dt / 2 (background at [nprims])
  // FP32-mixed walk: coordinates relative to (ymid, zmid) in units of K, so a
  // step is sqrt(-log2 u) (cos, sin) and the bridge test 2 d0 d1 <= dt (-ln U)
  // reads 2 d0 d1 <= -log2(U) / 2; walls at +-h
  float fhy, fhz;      // half-widths / K
  float fthr;          // 12.05 > 24 / 2, compared with 2 d0 d1 (FP32 uniforms are >= 2^-24)
  float fscr;          // fthr / 2, compared with d0 d1' in the per-step screen
  float fscr_root;     // least float r with fl(r r) > fscr: distances all > r pass both screens of a pair
  // generic signature: the phase of a full step in region r as the integer
  // cfx[r] = round(c[r] 2^phase_shift) (the largest in [2^29, 2^30]), summed
  // exactly in 64 bits along a path
  uint32_t cfx[kMaxRegions + 3];
  int32_t phase_shift;
  // model signature (which specialised region lookup the walkers use) and its
  // FP32 parameters in centred coordinates (units of K):
  //   kSigZ:    [z0]                      air above z0
  //   kSigZY:   [z0, y1]                  + half-space y < y1
  //   kSigZBox: [z0, y0, y1, zb0, zb1]    + box
  //   kSigZTri: [z0, A0,B0,C0, A1,B1,C1, A2,B2,C2]  + triangle, edges A a + B b + C
  //             (oriented: the interior is e >= 0 on all three)
  int32_t sig;
  // 1: finished paths record the phase and the exit point instead of the
  // weight (w_re = S at this request's frequency, w_im = tangential exit
  // coordinate), for weights at other frequencies computed afterwards
  uint32_t fanout;
  // step caps of the FP32 walk, which starts every pair of steps at an even
  // step index n: the pair is the last one when n >= cap2 (max_steps - 2, or
  // 0), and then its first step is the last allowed iff max_steps is odd;
  // the walker takes two pairs per iteration, and the second compares the
  // iteration's first n with cap2b (cap2 - 2, or 0)
  uint32_t cap2;
  uint32_t cap_odd;
  uint32_t cap2b;
  float sigp[12];
  // streams and limits
  uint32_t key0, key1;  // Philox key (seed low, high)
  uint32_t ctr3;        // 2 * stream
  uint32_t max_steps;
  uint32_t precision;   // 0 FP64, 1 FP32-mixed
  uint32_t n_tiles;
  uint32_t M;           // g_samples - 1
  uint32_t nprims;
  int32_t kind[kMaxPrims];
  double pd[kMaxPrims][6];    // FP64 geometry of the model's primitives
  // FP32 geometry relative to the centre in units of K: half-plane [c], box
  // [y0, y1, z0, z1], triangle its three edges as (A, B, C), edge k from
  // vertex k to vertex k + 1: e = fma(A, a, fma(B, b, C)), all three negated
  // for a clockwise triangle so that the interior is e >= 0
  float pf[kMaxPrims][kPfStride];
  const DevModel *model;      // resident model the primitives were taken from
  // sigma grid of the FP32 generic signature (null: the primitive loop); cell
  // (i, j) = (trunc(a gsy + goy), trunc(b gsz + goz)) clamped, at grid[j gy + i]
  const SigmaCell *grid;
  const SigmaCell *grid_ext;   // extension entries of the two-line cells
  uint32_t gy, gz;
  float gsy, goy, gsz, goz;
  float gmy, gmz;       // gy - 1, gz - 1: the cell index clamped in FP32
  // the grid's LDS form (kSigGenericLds): gy gz class bytes, then from byte
  // lds_table (a multiple of 16) the class table of SigmaCells; lds_bytes in
  // all (a multiple of 16)
  const uint8_t *lds_src;
  uint32_t lds_bytes, lds_table;
  const double *nodes;  // n x (y, z)
  const double *g;      // 4 x (M + 1) x (re, im)
  const DevTile *tiles;
  PathRec *recs;
  uint32_t *tile_counter;           // next tile to claim
  unsigned long long *done_counter; // paths completed (finished or capped)
  // served mode: walkers suspended by the previous slice (pool_in, resumed
  // first), tile remainders it left (extra_in, claimed before new tiles),
  // and where this slice suspends its own (pool_out, extra_out).
  const SuspRec *pool_in;
  SuspRec *pool_out;
  const DevTile *extra_in;
  DevTile *extra_out;
  uint32_t pool_in_n, extra_in_n;
  uint32_t pool_cap, extra_cap;     // capacity of pool_out / extra_out
  uint32_t *slice_ctl;              // SliceCtl words
};


// Request descriptor of the discontinuous-kappa walk (one vertical interface
// y = y_if; side 0 is y < y_if, side 1 is y >= y_if).
struct KReq {
  double y_lo, y_hi, z_lo, z_hi, y_if;
  double dt;
  double kdt[2];       // kappa_i dt
  double s[2];         // sqrt(kappa_i dt): step scale and interface disc radius
  double thr[2];       // 22.9 kappa_i dt: draw a bridge uniform only if 2 d0 d1 <= thr
  double p[2];         // kappa_i / (kappa_0 + kappa_1): resume on side i
  double kappa[2];
  double lre[2], lim[2];   // killing rate per side
  const double *g;     // 4 x (M + 1) x (re, im)
  const double *nodes; // n_nodes x (y, z)
  const DevTile *tiles;
  PathRec *recs;
  uint32_t *tile_counter;
  uint32_t n_tiles, M, key0, key1, ctr3, max_steps;
  uint32_t equal_kappa;   // kappa_0 == kappa_1: no interface rule
  uint32_t pad;
  // FP32-mixed walk: positions relative to (ymid, zmid)
  double ymid, zmid;
  float fhy, fhz;      // half-widths
  float fa_if;         // interface y_if - ymid
  float fdt, frdt;     // dt, 1 / dt
  float fK[2];         // sqrt(kappa_i dt) sqrt(2 ln 2): step length per sqrt(-log2 u)
  float fs[2];         // sqrt(kappa_i dt): disc radius
  float fthr[2];       // 16.7 kappa_i dt (FP32 uniforms are >= 2^-24)
  float fkdt[2];       // kappa_i dt
  float fkappa[2];
  float fp[2];         // kappa_i / (kappa_0 + kappa_1)
  float fpad;
};

}  // namespace sdd
