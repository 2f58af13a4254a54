// Device-side definitions shared by the liblbm kernels: lattices, PDF storage
// forms, tile records and kernel arguments.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
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

// ---- MRT moment bases (Eq. 8) -------------------------------------------------
// The paper does not give the MRT collision matrix; it is taken diagonal in
// the published orthogonal moment bases, Lallemand & Luo (2000) for D2Q9 and
// d'Humieres et al. (2002) for D3Q19, written here as integer polynomials in
// the velocity c.  Each moment relaxes with the rate of its class.
enum MrtClass : int { kMrtCons = 0, kMrtE, kMrtEps, kMrtQ, kMrtNu, kMrtPi, kMrtM, kMrtClasses };

struct MrtRow {
  int value;
  int cls;
};

// D2Q9: rho, e, eps, jx, qx, jy, qy, pxx, pxy.
constexpr MrtRow mrt_row9(int k, int x, int y) {
  const int c2 = x * x + y * y;
  switch (k) {
    case 0: return {1, kMrtCons};
    case 1: return {3 * c2 - 4, kMrtE};
    case 2: return {(8 - 21 * c2 + 9 * c2 * c2) / 2, kMrtEps};
    case 3: return {x, kMrtCons};
    case 4: return {(3 * c2 - 5) * x, kMrtQ};
    case 5: return {y, kMrtCons};
    case 6: return {(3 * c2 - 5) * y, kMrtQ};
    case 7: return {x * x - y * y, kMrtNu};
    default: return {x * y, kMrtNu};
  }
}

// D3Q19: rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy,
// pyz, pxz, mx, my, mz.
constexpr MrtRow mrt_row19(int k, int x, int y, int z) {
  const int c2 = x * x + y * y + z * z;
  switch (k) {
    case 0: return {1, kMrtCons};
    case 1: return {19 * c2 - 30, kMrtE};
    case 2: return {(21 * c2 * c2 - 53 * c2 + 24) / 2, kMrtEps};
    case 3: return {x, kMrtCons};
    case 4: return {(5 * c2 - 9) * x, kMrtQ};
    case 5: return {y, kMrtCons};
    case 6: return {(5 * c2 - 9) * y, kMrtQ};
    case 7: return {z, kMrtCons};
    case 8: return {(5 * c2 - 9) * z, kMrtQ};
    case 9: return {3 * x * x - c2, kMrtNu};
    case 10: return {(3 * c2 - 5) * (3 * x * x - c2), kMrtPi};
    case 11: return {y * y - z * z, kMrtNu};
    case 12: return {(3 * c2 - 5) * (y * y - z * z), kMrtPi};
    case 13: return {x * y, kMrtNu};
    case 14: return {y * z, kMrtNu};
    case 15: return {x * z, kMrtNu};
    case 16: return {(y * y - z * z) * x, kMrtM};
    case 17: return {(z * z - x * x) * y, kMrtM};
    default: return {(x * x - y * y) * z, kMrtM};
  }
}

template <class L>
constexpr MrtRow mrt_row(int k, int i) {
  if constexpr (L::Q == 9)
    return mrt_row9(k, L::C[i][0], L::C[i][1]);
  else
    return mrt_row19(k, L::C[i][0], L::C[i][1], L::C[i][2]);
}

template <class L>
constexpr int mrt_norm(int k) {
  int n = 0;
  for (int i = 0; i < L::Q; ++i) n += mrt_row<L>(k, i).value * mrt_row<L>(k, i).value;
  return n;
}

// Every moment of the basis is a polynomial in c of one parity: an even row
// takes the same value on c and -c, an odd row opposite values.  Returns
// +1 (even), -1 (odd) or 0 (neither; no row of the bases is).
template <class L>
constexpr int mrt_parity(int k) {
  bool even = true, odd = true;
  for (int i = 0; i < L::Q; ++i) {
    const int a = mrt_row<L>(k, i).value, b = mrt_row<L>(k, L::Opp[i]).value;
    even = even && a == b;
    odd = odd && a == -b;
  }
  return even ? 1 : odd ? -1 : 0;
}

// The p-th pair of opposite moving directions (i, opp(i)) with i < opp(i).
template <class L>
constexpr int pair_dir(int p) {
  for (int i = 1, n = 0; i < L::Q; ++i)
    if (i < L::Opp[i] && n++ == p) return i;
  return -1;
}

// Per class: -s and 1 - s/2 (FP64 and FP32).  Shear stress: s = 1/tau;
// conserved moments: s = 1 (the density's relaxation term vanishes and the
// momentum's cancels against the half-force shift of u).
struct MrtRates {
  double ms[kMrtClasses], mh[kMrtClasses];
  float msf[kMrtClasses], mhf[kMrtClasses];
};

// Moving wall (the lid of a driven cavity) on the face of a non-periodic axis
// beyond the last node (side 1) or before the first (side 0): a pull from
// beyond that face returns the bounce-back value plus corr_i =
// 6 w_i rho_w (c_i . u_w) (Ladd's moving-wall rule).  axis < 0: no lid.
struct LidArgs {
  int32_t axis;
  int32_t side;
  double corr[19];
  float corrf[19];
};

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
  // the stored bits as loaded, and their value (the shuffle step moves raw
  // values between lanes and converts each once)
  using Raw = double;
  __device__ static __forceinline__ Raw load_raw(const T *p, int64_t i) { return p[i]; }
  __device__ static __forceinline__ R value(Raw r, float) { return r; }
};

template <>
struct Store<LBM_F32_OFFSET> {
  using T = float;
  using R = float;
  static constexpr bool offset = true;
  __device__ static __forceinline__ R load(const T *p, int64_t i, float) { return p[i]; }
  __device__ static __forceinline__ void store(T *p, int64_t i, R v, float) { p[i] = v; }
  __device__ static __forceinline__ void store_nt(T *p, int64_t i, R v, float) { __builtin_nontemporal_store(v, p + i); }
  using Raw = float;
  __device__ static __forceinline__ Raw load_raw(const T *p, int64_t i) { return p[i]; }
  __device__ static __forceinline__ R value(Raw r, float) { return r; }
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
  // binary16 bits in the low half of a 32-bit register
  using Raw = uint32_t;
  __device__ static __forceinline__ Raw load_raw(const T *p, int64_t i) {
    return reinterpret_cast<const uint16_t *>(p)[i];
  }
  __device__ static __forceinline__ R value(Raw r, float inv) {
    return __half2float(__builtin_bit_cast(__half, (uint16_t)r)) * inv;
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
  MrtRates mrt;            // relaxation of the MRT collision
  LidArgs lid;             // moving wall on one face of the box
};

// The density that multiplies the velocity terms of the equilibrium and the
// force: rho in the quasi-compressible model, Eqs. (3) and (5); the reference
// density 1 in the incompressible model, Eqs. (4) and (6).
template <bool INC, class R>
__device__ __forceinline__ R velocity_density(R rho) {
  if constexpr (INC) return R(1);
  else return rho;
}

// Workgroup -> logical block remaps.  The hardware hands workgroups to the 8
// XCDs round-robin.  xcd_remap gives each XCD one contiguous range of blocks
// (and so of tiles), keeping neighbour tiles inside one XCD's L2.
// xcd_chunk gives XCD k the chunks k, k+8, k+16, ... of C consecutive blocks:
// neighbours stay together within a chunk while all XCDs stream through
// neighbouring memory at the same time (blocks past the last whole round of
// 8 C keep their index, so the map stays a bijection).
__device__ __forceinline__ int64_t xcd_chunk(int64_t b, int64_t nb, int64_t C) {
  const int64_t full = nb / (8 * C) * (8 * C);
  if (b >= full) return b;
  const int64_t k = b & 7, i = b >> 3;
  return ((i / C) * 8 + k) * C + i % C;
}

__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
  const int64_t k = b & 7, q = nb >> 3, r = nb & 7;
  return k * q + (k < r ? k : r) + (b >> 3);
}

// MRT collision, Eq. (8) with Guo forcing, in place on f (the PDFs, or their
// offsets f_i - w_i rho0 in the offset forms):
//   f* = f + M^-1 [-S M (f - f_eq) + (I - S/2) M F],
// f_eq from Eq. (3) or (4), u with the half-force shift; the rows of M are
// orthogonal, so M^-1 = M^T diag(1/norm).  With every rate 1/tau this is the
// BGK collision.
// c.v for a lattice velocity c with components in {-1, 0, 1}, without
// multiplications (IEEE rules keep 0 * v, so a plain dot product would not
// fold).
template <int CX, int CY, int CZ, class R>
__device__ __forceinline__ R cdot(R x, R y, R z) {
  R r = R(0);
  bool first = true;
  auto add = [&](int c, R v) {
    if (c == 0) return;
    const R t = c > 0 ? v : -v;
    r = first ? t : r + t;
    first = false;
  };
  add(CX, x);
  add(CY, y);
  add(CZ, z);
  return r;
}

// Moments of the Guo source F_i = w_i m [3 (c_i - u).g + 9 (c_i.u)(c_i.g)]
// in closed form: for a row P_k of the basis,
//   sum_i P_k(c_i) F_i = m [3 sum_a A_a g_a - 3 B (u.g) + 9 sum_ab C_ab u_a g_b]
// with the lattice sums B = sum_i w_i P_k(c_i), A_a = sum_i w_i P_k(c_i) c_ia
// and C_ab = sum_i w_i P_k(c_i) c_ia c_ib (compile-time constants, most of
// them zero), so the source never has to be formed per direction.
template <class L>
constexpr double mrt_src_B(int k) {
  double s = 0.0;
  for (int i = 0; i < L::Q; ++i) s += L::Wt[i] * mrt_row<L>(k, i).value;
  return s;
}
template <class L>
constexpr double mrt_src_A(int k, int a) {
  double s = 0.0;
  for (int i = 0; i < L::Q; ++i) s += L::Wt[i] * mrt_row<L>(k, i).value * L::C[i][a];
  return s;
}
template <class L>
constexpr double mrt_src_C(int k, int a, int b) {
  double s = 0.0;
  for (int i = 0; i < L::Q; ++i) s += L::Wt[i] * mrt_row<L>(k, i).value * L::C[i][a] * L::C[i][b];
  return s;
}

template <class L, int K, class R>
__device__ __forceinline__ R mrt_source_moment(R m, const R (&u)[3], const R (&g)[3], R ug) {
  R acc = R(0);
  bool any = false;
  auto add = [&](R term) {
    acc = any ? acc + term : term;
    any = true;
  };
  static_for<3>([&](auto A) {
    constexpr int a = decltype(A)::value;
    constexpr double ca = 3.0 * mrt_src_A<L>(K, a);
    if constexpr (ca != 0.0) add(R(ca) * g[a]);
  });
  {
    constexpr double cb = -3.0 * mrt_src_B<L>(K);
    if constexpr (cb != 0.0) add(R(cb) * ug);
  }
  static_for<3>([&](auto A) {
    constexpr int a = decltype(A)::value;
    static_for<3>([&](auto B) {
      constexpr int b = decltype(B)::value;
      constexpr double cc = 9.0 * mrt_src_C<L>(K, a, b);
      if constexpr (cc != 0.0) add(R(cc) * (u[a] * g[b]));
    });
  });
  return any ? m * acc : R(0);
}

template <class L, int S, bool INC, class R>
__device__ __forceinline__ void collide_mrt(R (&f)[L::Q], R sum, R jx, R jy, R jz, R rho0, R gx, R gy, R gz,
                                            const MrtRates &mr) {
  // Every multiply-add is an explicit fma and nothing else is contracted, so
  // each kernel variant (phase, launch mode) rounds the same way and the
  // single-copy steps stay bit-identical to the two-copy step.  sum and j
  // are plain sums of the gathered values.
#pragma clang fp contract(off)
  constexpr int Q = L::Q;
  constexpr bool off = Store<S>::offset;
  const R rho = off ? rho0 + sum : sum;
  const R m = velocity_density<INC>(rho);
  R ux, uy, uz;  // Eq. (5) or (6) with the half-force shift
  if constexpr (INC) {
    ux = std::fma(R(0.5), gx, jx);
    uy = std::fma(R(0.5), gy, jy);
    uz = std::fma(R(0.5), gz, jz);
  } else {
    const R inv = R(1) / rho;
    ux = std::fma(jx, inv, R(0.5) * gx);
    uy = std::fma(jy, inv, R(0.5) * gy);
    uz = std::fma(jz, inv, R(0.5) * gz);
  }
  const R uu = std::fma(ux, ux, std::fma(uy, uy, uz * uz));
  const R ug = std::fma(ux, gx, std::fma(uy, gy, uz * gz));
  const R uv[3] = {ux, uy, uz}, gv[3] = {gx, gy, gz};
  // The transforms work on pair sums and differences: an even row reads
  // d_i + d_opp(i) (and the rest direction), an odd row d_i - d_opp(i), so
  // each row takes half the terms; the inverse collects the even and odd rows'
  // contributions per pair and splits them back over the two directions.
  constexpr int P = (Q - 1) / 2;
  R ds[P], dd[P], ev[P], od[P];
  auto dev = [&](auto I) -> R {
    constexpr int i = decltype(I)::value;
    constexpr int cx = L::C[i][0], cy = L::C[i][1], cz = L::C[i][2];
    constexpr R w = (R)L::Wt[i];
    // c has components in {-1, 0, 1}: signed sums of the nonzero terms
    const R cu = cdot<cx, cy, cz>(ux, uy, uz);
    const R poly = std::fma(R(3), cu, std::fma(R(4.5) * cu, cu, R(-1.5) * uu));
    // f - f_eq, with f_eq (or its offset) w (rho + m poly), w (drho + m poly)
    return f[i] - w * std::fma(m, poly, off ? sum : rho);
  };
  const R d0 = dev(std::integral_constant<int, 0>{});
  static_for<P>([&](auto Pc) {
    constexpr int p = decltype(Pc)::value;
    constexpr int i = pair_dir<L>(p), j = L::Opp[i];
    const R di = dev(std::integral_constant<int, i>{}), dj = dev(std::integral_constant<int, j>{});
    ds[p] = di + dj;
    dd[p] = di - dj;
    ev[p] = R(0);
    od[p] = R(0);
  });
  R e0 = 0;
  // x + c v for an integer coefficient c, with the unit cases as plain adds
  auto madd = [](auto Cc, R v, R x) -> R {
    constexpr int c = decltype(Cc)::value;
    if constexpr (c == 1) return x + v;
    else if constexpr (c == -1) return x - v;
    else return std::fma(R(c), v, x);
  };
  static_for<Q>([&](auto K) {
    constexpr int k = decltype(K)::value;
    constexpr int par = mrt_parity<L>(k);
    static_assert(par != 0, "every moment of the basis is even or odd in c");
    constexpr int c0 = mrt_row<L>(k, 0).value;  // zero in every odd row
    R dm = 0;
    if constexpr (c0 != 0) dm = madd(std::integral_constant<int, c0>{}, d0, dm);
    static_for<P>([&](auto Pc) {
      constexpr int p = decltype(Pc)::value;
      constexpr int c = mrt_row<L>(k, pair_dir<L>(p)).value;
      if constexpr (c != 0) dm = madd(std::integral_constant<int, c>{}, par > 0 ? ds[p] : dd[p], dm);
    });
    const R fm = mrt_source_moment<L, k>(m, uv, gv, ug);
    constexpr int cl = mrt_row<L>(k, 0).cls;
    constexpr R inv = R(1.0 / mrt_norm<L>(k));
    R ms, mh;
    if constexpr (sizeof(R) == 8) {
      ms = (R)mr.ms[cl];
      mh = (R)mr.mh[cl];
    } else {
      ms = (R)mr.msf[cl];
      mh = (R)mr.mhf[cl];
    }
    const R y = std::fma(ms, dm, mh * fm) * inv;
    if constexpr (c0 != 0) e0 = madd(std::integral_constant<int, c0>{}, y, e0);
    static_for<P>([&](auto Pc) {
      constexpr int p = decltype(Pc)::value;
      constexpr int c = mrt_row<L>(k, pair_dir<L>(p)).value;
      if constexpr (c != 0) {
        if constexpr (par > 0)
          ev[p] = madd(std::integral_constant<int, c>{}, y, ev[p]);
        else
          od[p] = madd(std::integral_constant<int, c>{}, y, od[p]);
      }
    });
  });
  f[0] = f[0] + e0;
  static_for<P>([&](auto Pc) {
    constexpr int p = decltype(Pc)::value;
    constexpr int i = pair_dir<L>(p), j = L::Opp[i];
    f[i] = f[i] + (ev[p] + od[p]);
    f[j] = f[j] + (ev[p] - od[p]);
  });
}

}  // namespace lbm
