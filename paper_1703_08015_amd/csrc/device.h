// Device-side definitions shared by the liblbm kernels: lattices, PDF storage
// forms, tile records and kernel arguments.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

#include "lbm.h"

namespace lbm {

// ---- lattices --------------------------------------------------------------
// Standard D2Q9 and D3Q19 velocity sets; weights of the equilibrium, Eq. (3),
// with c_s^2 = 1/3.  Opposite pairs are adjacent: (1,2), (3,4), ...
struct D2Q9 {
  static constexpr int Q = 9;
  static constexpr int C[9][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                                  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
  static constexpr double Wt[9] = {4.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9, 1.0 / 9,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  static constexpr int Opp[9] = {0, 2, 1, 4, 3, 6, 5, 8, 7};
};

struct D3Q19 {
  static constexpr int Q = 19;
  static constexpr int C[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                                   {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                                   {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                   {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
  static constexpr double Wt[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  static constexpr int Opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
};

// Lane regions of the scalar-mask D3Q19 step (4x4x4 tiles): for direction i
// (1..18) region w = 0 holds the lanes whose source x - c_i lies in the tile
// itself, region w = 1..7 those whose source wraps across the axes flagged by
// the bits of w (only axes with c_a != 0).  The planner stores, per tile, the
// base entry index of every (i, w) region in this order; the kernel adds the
// source's rank.  60 regions, padded to 64.
constexpr int kRegionBases = 64;

constexpr bool region_valid(int i, int w) {
  const int cx = D3Q19::C[i][0], cy = D3Q19::C[i][1], cz = D3Q19::C[i][2];
  return w == 0 || ((!(w & 1) || cx) && (!((w >> 1) & 1) || cy) && (!((w >> 2) & 1) || cz));
}

constexpr int region_index(int i, int w) {
  int n = 0;
  for (int a = 1; a < 19; ++a)
    for (int b = 0; b < 8; ++b) {
      if (a == i && b == w) return n;
      if (region_valid(a, b)) ++n;
    }
  return -1;
}

// Step phases: the two-copy step (source and destination buffers differ), or
// one of the two in-place steps of the single-copy form: the gather/scatter
// step that follows init or a local step (whose state holds f*_i in slot
// opp(i)), and the local step that follows it (whose state holds the
// streamed f_i in slot i).
enum StepPhase : int { kPhaseTwoCopy = 0, kPhaseAAGather = 1, kPhaseAALocal = 2 };

// PDF pointers of a step: restrict-qualified when source and destination are
// distinct buffers (two-copy), plain in place.
template <int PH, class T>
using in_ptr = std::conditional_t<PH == kPhaseTwoCopy, const T *__restrict__, const T *>;
template <int PH, class T>
using out_ptr = std::conditional_t<PH == kPhaseTwoCopy, T *__restrict__, T *>;

// Compile-time loop: f(std::integral_constant<int, I>) for I = 0..N-1.
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// ---- storage forms -----------------------------------------------------------
// F64: the PDF itself.  F32/F16: the offset f_i - w_i rho0 (FP16 scaled by
// 2^s), so that the stored values carry the deviation from rest rather than
// the large constant w_i rho0.
template <int S>
struct Store;

template <>
struct Store<LBM_F64> {
  using T = double;      // stored element
  using R = double;      // arithmetic type of the step
  static constexpr bool offset = false;
  __device__ static __forceinline__ R load(const T *p, int64_t i, float) { return p[i]; }
  __device__ static __forceinline__ void store(T *p, int64_t i, R v, float) { p[i] = v; }
  __device__ static __forceinline__ void store_nt(T *p, int64_t i, R v, float) { __builtin_nontemporal_store(v, p + i); }
};

template <>
struct Store<LBM_F32_OFFSET> {
  using T = float;
  using R = float;
  static constexpr bool offset = true;
  __device__ static __forceinline__ R load(const T *p, int64_t i, float) { return p[i]; }
  __device__ static __forceinline__ void store(T *p, int64_t i, R v, float) { p[i] = v; }
  __device__ static __forceinline__ void store_nt(T *p, int64_t i, R v, float) { __builtin_nontemporal_store(v, p + i); }
};

template <>
struct Store<LBM_F16_OFFSET> {
  using T = __half;
  using R = float;
  static constexpr bool offset = true;
  // inv / scale are exact powers of two, so scaling is exact barring over/underflow
  __device__ static __forceinline__ R load(const T *p, int64_t i, float inv) { return __half2float(p[i]) * inv; }
  __device__ static __forceinline__ void store(T *p, int64_t i, R v, float scale) {
    p[i] = __float2half_rn(v * scale);
  }
  __device__ static __forceinline__ void store_nt(T *p, int64_t i, R v, float scale) {
    const __half h = __float2half_rn(v * scale);
    __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, h), reinterpret_cast<uint16_t *>(p) + i);
  }
};

// ---- tables ------------------------------------------------------------------
// Per non-empty tile: first PDF entry of its region and fluid-node count.  The
// region holds q blocks of n entries (direction-major), entry i*n + r being
// direction i of the r-th non-solid node in lane order; regions start on
// 128-byte boundaries.
struct TileRec {
  int64_t off;     // first PDF entry
  int32_t n;       // non-solid nodes
  int32_t sample;  // sample index (batches)
};

struct SampleRec {
  double g[3];      // body acceleration
  int64_t dense0;   // first node in concatenated dense arrays
  int64_t n_nodes;  // nx*ny*nz
  int64_t tile0;    // first tile
  int64_t n_ftiles; // tiles of this sample
  int64_t nbase0;   // first fluid node (compact numbering)
  int64_t n_fluid;  // fluid nodes of this sample
  int32_t shape[3]; // nx, ny, nz
  int32_t frozen;   // 1: out of the active list (single copy: its state is in layout 0)
};

// Compact record of a tile for the scalar-mask D3Q19 kernel: region offset,
// fluid-node count and fluid mask in one 16-byte scalar load.  Index n_ftiles
// is an all-solid sentinel that empty neighbours point at.
struct NbRec {
  uint32_t off;
  uint32_t n;
  uint64_t mask;
  int32_t sample;
  int32_t pad;
};

// Per-sample collision constants of the D3Q19 step (host-prepared):
// a_i = 3w + 9(1 - w/2) c_i.g and b_i = 3(1 - w/2) c_i.g, w = 1/tau.
struct CollideCoef {
  double g[3];
  double omega;
  double a[19], b[19];
  float af[19], bf[19];
};

// Arguments shared by the per-tile kernels.
struct TileArgs {
  const TileRec *rec;
  const uint64_t *fluid;   // words per tile
  const int32_t *pre;      // per tile and word: fluid nodes in earlier words
  const int32_t *nbr;      // 27 per tile
  const int32_t *coord;    // 3 per tile
  const int64_t *nbase;    // first compact fluid-node index of each tile
  const SampleRec *samples;
  int64_t n_waves;         // non-empty tiles * words
  int64_t n_fluid;
  double rho0;
  float f16_scale;         // 2^s
  float f16_inv;           // 2^-s
  int32_t model;           // LBM_MODEL_*
  int32_t aa_phase;        // -1: two copies; single copy: layout of the state (0 or 1, see kernels.hip)
};

// The density that multiplies the velocity terms of the equilibrium and the
// force: rho in the quasi-compressible model, Eqs. (3) and (5); the reference
// density 1 in the incompressible model, Eqs. (4) and (6).
template <bool INC, class R>
__device__ __forceinline__ R velocity_density(R rho) {
  if constexpr (INC) return R(1);
  else return rho;
}

// Workgroup -> logical block remap: the hardware hands workgroups to the 8
// XCDs round-robin; this gives each XCD one contiguous range of blocks (and
// so of tiles), keeping neighbour tiles inside one XCD's L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
  const int64_t k = b & 7, q = nb >> 3, r = nb & 7;
  return k * q + (k < r ? k : r) + (b >> 3);
}

}  // namespace lbm
