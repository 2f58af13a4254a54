// D3Q19 fused step on 4x4x4 tiles, one wavefront per tile, with all tile
// bookkeeping on the scalar unit.
//
// Gather (two-copy method, Sec. 3, Fig. 5): lane l = x + 4y + 16z pulls f_i
// from the node l - c_i.  For a direction i the lanes fall into at most four
// regions by which axes the source wraps across: the tile itself, the face
// neighbours and the edge neighbour (D3Q19 has no corner directions).  In a
// region whose tile has fluid mask M, the source lane is s = l - d for a
// constant shift d, so shifting M by d on the scalar unit turns
//   "is the source non-solid"   into bit l of the shifted mask, and
//   "rank of the source"        into v_mbcnt of the shifted mask (number of
//                                set bits below lane l), plus a scalar
//                                correction for bits shifted out below 0.
// Two v_mbcnt give a region's entry index; regions and the half-way
// bounce-back (Sec. 3.2: propagation only between non-solid nodes) are merged
// with v_cndmask on scalar lane masks.  Neighbour records (region offset,
// node count, fluid mask) come through scalar loads; nothing is staged in LDS
// and there is no barrier.
//
// Shuffle form (two-copy step only): every lane first loads its own node's
// 19 post-collision values with coalesced loads (the tile's direction blocks
// are contiguous in rank order).  A source inside the tile is then another
// lane of the same wavefront, so lane l takes f*_i(l - c_i) from lane
// l - d_i: a DPP row shift when c_i lies in a z-layer of 16 lanes, a
// ds_bpermute otherwise.  Only the lanes whose source lies in a neighbour
// tile still gather from memory, with the region arithmetic above restricted
// to the neighbour regions, and the half-way bounce-back takes the lane's own
// value of opp(i) from a register.
//
// Single-copy form (the in-place "AA" pattern, one PDF buffer): phase 1
// gathers f_i(x) from the post-collision value f*_i(x - c_i), which the
// previous step stored in the source node's slot opp(i) (its own slot i on a
// bounce-back), and writes f*_i(x) to the address that the same node read
// for opp(i), i.e. into slot i of x + c_i (slot opp(i) of x on a
// bounce-back).  Each entry is read and written by one node only, so the
// step is safe in place.  Phase 2 then reads f_i(x) from the node's own slot
// i and writes f*_i(x) to its own slot opp(i).  Two steps move the same
// bytes as two steps of the two-copy method.
//
// Collision (Eqs. 2 and 7 with Guo forcing; quasi-compressible Eqs. 3 and 5
// or incompressible Eqs. 4 and 6) is regrouped so that each direction costs
// four fused multiply-adds:
//   out_i = (1-w) f_i + w_i [P + m (b_i + cu_i (a_i + h cu_i))]
// with cu_i = c_i.u, h = 9w/2, a_i = 3w + 9(1-w/2) c_i.g, b_i = 3(1-w/2) c_i.g
// (per-sample constants prepared on the host), m the density of the velocity
// terms (rho, or 1 in the incompressible model) and, per node,
// P = w (rho - 3/2 m u.u) - 3(1-w/2) m u.g for the full form and
// P = w (drho - 3/2 m u.u) - 3(1-w/2) m u.g for the offset forms.
#include "device.h"
#include "kernels.h"

namespace lbm {
namespace {

// Lanes of a 4x4x4 tile whose source x - c wraps into a neighbour exactly
// along the axes flagged by (wx, wy, wz).
constexpr uint64_t region(int cx, int cy, int cz, int wx, int wy, int wz) {
  uint64_t m = 0;
  for (int l = 0; l < 64; ++l) {
    const int x = l & 3, y = (l >> 2) & 3, z = l >> 4;
    const bool ax = (cx > 0 && x == 0) || (cx < 0 && x == 3);
    const bool ay = (cy > 0 && y == 0) || (cy < 0 && y == 3);
    const bool az = (cz > 0 && z == 0) || (cz < 0 && z == 3);
    if (ax == (wx != 0) && ay == (wy != 0) && az == (wz != 0)) m |= 1ull << l;
  }
  return m;
}

template <int D>
__device__ __forceinline__ uint64_t shifted(uint64_t m) {
  if constexpr (D >= 0)
    return m << D;
  else
    return m >> (-D);
}

// set bits of m below -D (those a right shift by -D drops), 0 for D >= 0
template <int D>
__device__ __forceinline__ uint32_t dropped(uint64_t m) {
  if constexpr (D >= 0)
    return 0u;
  else
    return (uint32_t)__popcll(m & ((1ull << (-D)) - 1ull));
}

__device__ __forceinline__ uint32_t mbcnt(uint64_t x, uint32_t acc) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(x >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)x, acc));
}

// lanes set in the scalar mask take if_set, the others if_clear
__device__ __forceinline__ uint32_t select_lanes(uint64_t lanes, uint32_t if_set, uint32_t if_clear) {
  uint32_t r;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(if_clear), "v"(if_set), "s"(lanes));
  return r;
}

// Lane l receives x from lane l - d of the wavefront, d = cx + 4 cy + 16 cz
// the in-tile offset of direction c.  A direction within one z-layer (the 16
// lanes of a DPP row) is a row shift; one that crosses layers goes through
// ds_bpermute.  Lanes whose source l - d lies outside the tile receive an
// unspecified value (every such lane takes a neighbour's value instead).
template <int CX, int CY, int CZ>
__device__ __forceinline__ uint32_t lane_shift32(uint32_t x, int lane) {
  constexpr int d = CX + 4 * CY + 16 * CZ;
  if constexpr (d == 0) {
    return x;
  } else if constexpr (CZ == 0) {
    constexpr int ctrl = d > 0 ? 0x110 + d : 0x100 - d;  // row_shr:d / row_shl:-d
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, ctrl, 0xf, 0xf, true);
  } else {
    return (uint32_t)__builtin_amdgcn_ds_bpermute(((lane - d) & 63) << 2, (int)x);
  }
}

template <int CX, int CY, int CZ, class V>
__device__ __forceinline__ V lane_shift(V x, int lane) {
  if constexpr (sizeof(V) == 8) {
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint64_t lo = lane_shift32<CX, CY, CZ>((uint32_t)b, lane);
    const uint64_t hi = lane_shift32<CX, CY, CZ>((uint32_t)(b >> 32), lane);
    return __builtin_bit_cast(V, lo | hi << 32);
  } else {
    return __builtin_bit_cast(V, lane_shift32<CX, CY, CZ>(__builtin_bit_cast(uint32_t, x), lane));
  }
}

// lanes set in the scalar mask (used as a lane predicate)
__device__ __forceinline__ bool lane_in(uint64_t lanes) { return __builtin_amdgcn_inverse_ballot_w64(lanes); }

// The 18 neighbour slots a D3Q19 tile pulls from (6 faces, 12 edges; the
// 3x3x3 index k = (dx+1) + 3(dy+1) + 9(dz+1)), in the order of the compact
// neighbour row uploaded for this kernel.
constexpr int kSlots[18] = {4, 22, 10, 16, 12, 14, 1, 3, 5, 7, 9, 11, 15, 17, 19, 21, 23, 25};
constexpr int slot_of(int k) {
  for (int j = 0; j < 18; ++j)
    if (kSlots[j] == k) return j;
  return -1;
}

constexpr int kTwoCopy = kPhaseTwoCopy, kAAGather = kPhaseAAGather, kAALocal = kPhaseAALocal;

// One 4x4x4 tile: gather, collide, store.  Lanes of solid nodes return
// early (in the shuffle form SH after the shuffles); every value the
// wavefront branches on is uniform.
template <int S, bool NT, bool INC, int PH, bool MRT, bool SH>
__device__ __forceinline__ void step19_tile(int64_t tile, in_ptr<PH, void> src_, out_ptr<PH, void> dst_,
                                            const TileArgs &a, const NbRec *__restrict__ nrec,
                                            const uint32_t *__restrict__ nrow, const uint32_t *__restrict__ rbase,
                                            const CollideCoef *__restrict__ coef) {
  using L = D3Q19;
  using St = Store<S>;
  using T = typename St::T;
  using R = typename St::R;
  in_ptr<PH, T> src = static_cast<const T *>(src_);
  out_ptr<PH, T> dst = static_cast<T *>(dst_);
  const int lane = threadIdx.x & 63;

  // own record and the 18 neighbour records (empty neighbours point at an
  // all-solid sentinel record, so every load is unconditional); the local
  // phase of the single-copy form needs only its own
  const NbRec own = nrec[tile];
  NbRec nb[PH == kAALocal ? 1 : 18];
  if constexpr (PH != kAALocal)
    static_for<18>([&](auto J) {
      constexpr int j = decltype(J)::value;
      nb[j] = *reinterpret_cast<const NbRec *>(reinterpret_cast<const char *>(nrec) + nrow[tile * 20 + j]);
    });
  const uint64_t M = own.mask;
  static_assert(!SH || PH == kTwoCopy, "the shuffle form is a two-copy step");
  if constexpr (!SH)
    if (!((M >> lane) & 1ull)) return;
  const uint32_t ooff = own.off, on = own.n;
  const uint32_t rank = mbcnt(M, 0u);
  // FP16 reads each lane region's base entry from the planner's table; the
  // other forms compute it (off + b*n + fluid nodes shifted out below lane 0,
  // b the slot read: i, or opp(i) in the single-copy gather)
  constexpr bool kTable = S == LBM_F16_OFFSET && PH != kAALocal;
  const uint32_t *__restrict__ rb = kTable ? rbase + tile * kRegionBases : nullptr;

  R f[19];
  uint32_t ea[PH == kAAGather ? 19 : 1];  // entries read, rewritten by the single-copy gather
  if constexpr (SH) {
    using Raw = typename St::Raw;
    // own values, coalesced; a solid lane reads entry 0 of the tile (its value is never used)
    const uint32_t eo = lane_in(M) ? rank : 0u;
    Raw v[19], gv[19];
    static_for<19>([&](auto I) {
      constexpr int i = decltype(I)::value;
      v[i] = St::load_raw(src, (int64_t)(ooff + (uint32_t)i * on + eo));
    });
    gv[0] = v[0];
    static_for<18>([&](auto Im) {
      constexpr int i = decltype(Im)::value + 1;
      constexpr int cx = L::C[i][0], cy = L::C[i][1], cz = L::C[i][2];
      constexpr int d0 = cx + 4 * cy + 16 * cz;
      constexpr uint64_t R0 = region(cx, cy, cz, 0, 0, 0);
      Raw t = lane_shift<cx, cy, cz>(v[i], lane);
      uint64_t from_fluid = shifted<d0>(M) & R0, halo = 0;
      uint32_t e = ooff;  // lanes outside every neighbour region keep a valid, unused entry
      static_for<8>([&](auto Wc) {
        constexpr int w = decltype(Wc)::value;
        constexpr int wx = w & 1, wy = (w >> 1) & 1, wz = (w >> 2) & 1;
        if constexpr (w != 0 && (!wx || cx) && (!wy || cy) && (!wz || cz)) {
          constexpr uint64_t Rr = region(cx, cy, cz, wx, wy, wz);
          constexpr int dr = d0 - (wx ? 4 * cx : 0) - (wy ? 16 * cy : 0) - (wz ? 64 * cz : 0);
          constexpr int k = 13 + (wx ? -cx : 0) + 3 * (wy ? -cy : 0) + 9 * (wz ? -cz : 0);
          const NbRec &r = nb[slot_of(k)];
          const uint64_t Xr = shifted<dr>(r.mask);
          halo |= Xr & Rr;
          uint32_t base;
          if constexpr (kTable)
            base = rb[region_index(i, w)];
          else
            base = r.off + (uint32_t)i * r.n + dropped<dr>(r.mask);
          e = select_lanes(Rr, mbcnt(Xr, base), e);
        }
      });
      from_fluid |= halo;
      // only lanes whose source is a non-solid node of a neighbour tile load
      if (lane_in(halo)) t = St::load_raw(src, (int64_t)e);
      // half-way bounce-back: the lane's own post-collision value opp(i)
      gv[i] = lane_in(from_fluid) ? t : v[L::Opp[i]];
    });
    if (!lane_in(M)) return;
    static_for<19>([&](auto I) {
      constexpr int i = decltype(I)::value;
      f[i] = St::value(gv[i], a.f16_inv);
    });
  } else
  static_for<19>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = L::C[i][0], cy = L::C[i][1], cz = L::C[i][2];
    constexpr int ib = PH == kAAGather ? L::Opp[i] : i;  // slot of the source's value
    if constexpr (i == 0 || PH == kAALocal) {
      f[i] = St::load(src, (int64_t)(ooff + (uint32_t)i * on + rank), a.f16_inv);
      if constexpr (PH == kAAGather) ea[0] = ooff + rank;
    } else {
      constexpr int d0 = cx + 4 * cy + 16 * cz;
      constexpr uint64_t R0 = region(cx, cy, cz, 0, 0, 0);
      const uint64_t X0 = shifted<d0>(M);
      uint64_t from_fluid = X0 & R0;
      constexpr int ri0 = region_index(i, 0);
      uint32_t e;
      if constexpr (kTable)
        e = mbcnt(X0, rb[ri0]);
      else
        e = mbcnt(X0, ooff + (uint32_t)ib * on + dropped<d0>(M));
      static_for<8>([&](auto Wc) {
        constexpr int w = decltype(Wc)::value;
        constexpr int wx = w & 1, wy = (w >> 1) & 1, wz = (w >> 2) & 1;
        if constexpr (w != 0 && (!wx || cx) && (!wy || cy) && (!wz || cz)) {
          constexpr uint64_t Rr = region(cx, cy, cz, wx, wy, wz);
          constexpr int dr = d0 - (wx ? 4 * cx : 0) - (wy ? 16 * cy : 0) - (wz ? 64 * cz : 0);
          constexpr int k = 13 + (wx ? -cx : 0) + 3 * (wy ? -cy : 0) + 9 * (wz ? -cz : 0);
          const NbRec &r = nb[slot_of(k)];
          const uint64_t Xr = shifted<dr>(r.mask);
          from_fluid |= Xr & Rr;
          constexpr int riw = region_index(i, w);
          uint32_t base;
          if constexpr (kTable)
            base = rb[riw];
          else
            base = r.off + (uint32_t)ib * r.n + dropped<dr>(r.mask);
          e = select_lanes(Rr, mbcnt(Xr, base), e);
        }
      });
      // half-way bounce-back: a solid or missing source returns the node's own
      // post-collision value opp(i), held in slot opp(i) (slot i in place)
      constexpr int bb = PH == kAAGather ? i : L::Opp[i];
      e = select_lanes(from_fluid, e, ooff + (uint32_t)bb * on + rank);
      f[i] = St::load(src, (int64_t)e, a.f16_inv);
      if constexpr (PH == kAAGather) ea[i] = e;
      // FP64 and FP32 two-copy BGK: keep each load where its address is
      // ready, so the wavefront's loads overlap its own remaining address
      // work instead of waiting for all 19 addresses (+1% FP64, +3-4% FP32
      // measured; FP16, whose table reads then stop batching, would lose half
      // its rate)
      if constexpr (S != LBM_F16_OFFSET && PH == kTwoCopy && !MRT) __builtin_amdgcn_sched_barrier(0);
    }
  });
  const CollideCoef &cc = coef[own.sample];
  // two-copy: own slot i of the other buffer; single-copy gather: where
  // opp(i) was read; single-copy local: own slot opp(i)
  auto put = [&](auto I, R out) {
    constexpr int i = decltype(I)::value;
    T *blk;
    uint32_t e;
    if constexpr (PH == kTwoCopy) {
      blk = dst + (ooff + (uint32_t)i * on);
      e = rank;
    } else if constexpr (PH == kAAGather) {
      blk = dst;
      e = ea[L::Opp[i]];
    } else {
      blk = dst;
      e = ooff + (uint32_t)L::Opp[i] * on + rank;
    }
    if constexpr (NT)
      St::store_nt(blk, (int64_t)e, out, a.f16_scale);
    else
      St::store(blk, (int64_t)e, out, a.f16_scale);
  };
  R sum = 0, jx = 0, jy = 0, jz = 0;
  static_for<19>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = L::C[i][0], cy = L::C[i][1], cz = L::C[i][2];
    sum += f[i];
    if constexpr (cx > 0) jx += f[i];
    if constexpr (cx < 0) jx -= f[i];
    if constexpr (cy > 0) jy += f[i];
    if constexpr (cy < 0) jy -= f[i];
    if constexpr (cz > 0) jz += f[i];
    if constexpr (cz < 0) jz -= f[i];
  });
  const R gx = (R)cc.g[0], gy = (R)cc.g[1], gz = (R)cc.g[2];
  if constexpr (MRT) {
    // Eq. (8) in the orthogonal moment basis
    collide_mrt<L, S, INC>(f, sum, jx, jy, jz, (R)a.rho0, gx, gy, gz, a.mrt);
    static_for<19>([&](auto I) { put(I, f[decltype(I)::value]); });
    return;
  }
  {
  // Every multiply-add below is an explicit fma and nothing else is
  // contracted, so the two-copy step and both single-copy phases round
  // identically whatever the surrounding code lets the compiler fuse.
#pragma clang fp contract(off)
  const R om = (R)cc.omega, om1 = R(1) - om, fo = std::fma(R(-0.5), om, R(1)), h = R(4.5) * om;
  const R rho = St::offset ? (R)a.rho0 + sum : sum;
  const R m = velocity_density<INC>(rho);
  R ux, uy, uz;
  if constexpr (INC) {
    ux = std::fma(R(0.5), gx, jx), uy = std::fma(R(0.5), gy, jy), uz = std::fma(R(0.5), gz, jz);
  } else {
    const R inv = R(1) / rho;
    ux = std::fma(jx, inv, R(0.5) * gx), uy = std::fma(jy, inv, R(0.5) * gy), uz = std::fma(jz, inv, R(0.5) * gz);
  }
  const R uu = std::fma(ux, ux, std::fma(uy, uy, uz * uz));
  const R ug = std::fma(ux, gx, std::fma(uy, gy, uz * gz));
  R P;
  if constexpr (INC)
    P = std::fma(om, std::fma(R(-1.5), uu, St::offset ? sum : rho), -(R(3) * fo) * ug);
  else if constexpr (St::offset)
    P = std::fma(om, std::fma(R(-1.5) * rho, uu, sum), -(R(3) * fo * rho) * ug);
  else
    P = std::fma(om * rho, std::fma(R(-1.5), uu, R(1)), -(R(3) * fo * rho) * ug);
  const R wr1 = R(L::Wt[1]) * m, wr2 = R(L::Wt[7]) * m;
  const R wp1 = R(L::Wt[1]) * P, wp2 = R(L::Wt[7]) * P;

  static_for<19>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = L::C[i][0], cy = L::C[i][1], cz = L::C[i][2];
    R out;
    if constexpr (i == 0) {
      out = std::fma(om1, f[0], R(L::Wt[0]) * P);
    } else {
      const R cu = cdot<cx, cy, cz>(ux, uy, uz);
      const R ai = St::offset ? (R)cc.af[i] : (R)cc.a[i];
      const R bi = St::offset ? (R)cc.bf[i] : (R)cc.b[i];
      const R t2 = std::fma(cu, std::fma(h, cu, ai), bi);
      constexpr bool face = (cx != 0) + (cy != 0) + (cz != 0) == 1;
      out = std::fma(om1, f[i], std::fma(face ? wr1 : wr2, t2, face ? wp1 : wp2));
    }
    put(I, out);
  });
  }
}

// Which tiles a launch visits.
enum { kDirect = 0, kList = 1, kPersistent = 2 };

// kDirect: wavefront w updates tile w.  kList: wavefront w updates tile
// list[w] if w < *count.  kPersistent: a fixed grid of G wavefronts strides
// over list[0 .. *count).  The count lives in device memory, so a captured
// graph stays valid when the active set changes.
template <int S, int WPB, bool NT, bool INC, int PH, bool MRT, int MODE, bool SH>
__global__ void __launch_bounds__(64 * WPB)
    k_step19(in_ptr<PH, void> src, out_ptr<PH, void> dst, TileArgs a, const NbRec *__restrict__ nrec,
             const uint32_t *__restrict__ nrow, const uint32_t *__restrict__ rbase,
             const CollideCoef *__restrict__ coef, const int32_t *__restrict__ list,
             const int32_t *__restrict__ count) {
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  // XCD assignment, chosen per form by measurement: chunks of 8 blocks for
  // the two-copy FP64/FP32 step (BGK and MRT), 16 for the FP64 BGK single
  // copy, one contiguous range per XCD for everything else (FP16, the other
  // single-copy forms and the persistent grid)
  constexpr int kChunk = MODE == kPersistent ? 0
                         : PH == kTwoCopy    ? (S == LBM_F16_OFFSET ? 0 : 8)
                                             : (S == LBM_F64 && !MRT ? 16 : 0);
  const int64_t blk = kChunk ? xcd_chunk(blockIdx.x, gridDim.x, kChunk) : xcd_remap(blockIdx.x, gridDim.x);
  const int64_t gw = blk * WPB + wv;
  if constexpr (MODE == kDirect) {
    if (gw >= a.n_waves) return;
    step19_tile<S, NT, INC, PH, MRT, SH>(gw, src, dst, a, nrec, nrow, rbase, coef);
  } else if constexpr (MODE == kList) {
    if (gw >= (int64_t)*count) return;
    step19_tile<S, NT, INC, PH, MRT, SH>(list[gw], src, dst, a, nrec, nrow, rbase, coef);
  } else {
    const int64_t n = *count, G = (int64_t)gridDim.x * WPB;
    for (int64_t k = gw; k < n; k += G)
      step19_tile<S, NT, INC, PH, MRT, SH>(list[k], src, dst, a, nrec, nrow, rbase, coef);
  }
}

template <int V>
using IC = std::integral_constant<int, V>;
template <bool V>
using BC = std::integral_constant<bool, V>;

// Calls f(storage, waves per block, model, phase, MRT, shuffle form) with
// compile-time constants.  The shuffle form exists for the two-copy step.
template <class F>
hipError_t with_variant(const Variant &v, int phase, bool shuffle, F &&f) {
  // MRT is built for 4 waves per workgroup only (the planner rejects others)
  auto by_collision = [&](auto s, auto w, auto inc, auto ph, auto sh) -> hipError_t {
    if constexpr (decltype(w)::value == 4)
      if (v.collision == LBM_COLLISION_MRT) return f(s, w, inc, ph, BC<true>{}, sh);
    return f(s, w, inc, ph, BC<false>{}, sh);
  };
  auto by_phase = [&](auto s, auto w, auto inc) -> hipError_t {
    switch (phase) {
      case kAAGather: return by_collision(s, w, inc, IC<kAAGather>{}, BC<false>{});
      case kAALocal: return by_collision(s, w, inc, IC<kAALocal>{}, BC<false>{});
      default:
        return shuffle ? by_collision(s, w, inc, IC<kTwoCopy>{}, BC<true>{})
                       : by_collision(s, w, inc, IC<kTwoCopy>{}, BC<false>{});
    }
  };
  auto by_model = [&](auto s, auto w) -> hipError_t {
    return v.model == LBM_MODEL_INCOMPRESSIBLE ? by_phase(s, w, BC<true>{}) : by_phase(s, w, BC<false>{});
  };
  auto by_wpb = [&](auto s) -> hipError_t {
    switch (v.wpb) {
      case 1: return by_model(s, IC<1>{});
      case 2: return by_model(s, IC<2>{});
      case 4: return by_model(s, IC<4>{});
      default: return by_model(s, IC<8>{});
    }
  };
  switch (v.storage) {
    case LBM_F64: return by_wpb(IC<LBM_F64>{});
    case LBM_F32_OFFSET: return by_wpb(IC<LBM_F32_OFFSET>{});
    default: return by_wpb(IC<LBM_F16_OFFSET>{});
  }
}

}  // namespace

// 4x4x4 tiles, or 4x4x8 tiles run as two 4x4x4 halves (one wavefront each)
// whose records the planner builds
bool step19_supported(const Variant &v) { return v.q == 19 && v.ax == 4 && v.ay == 4 && (v.az == 4 || v.az == 8); }

hipError_t launch_step19(const Variant &v, int phase, bool shuffle, const void *src, void *dst, const TileArgs &a,
                         const NbRec *nrec, const uint32_t *nrow, const uint32_t *rbase, const CollideCoef *coef,
                         bool nontemporal, const int32_t *list, const int32_t *count, int mode,
                         int64_t blocks_persistent, hipStream_t s) {
  if (a.n_waves == 0) return hipSuccess;
  if ((phase == kTwoCopy) == (src == dst)) return hipErrorInvalidValue;  // in place exactly for the single copy
  if (shuffle && phase != kTwoCopy) return hipErrorInvalidValue;
  const unsigned blocks =
      mode == kPersistent ? (unsigned)blocks_persistent : (unsigned)((a.n_waves + v.wpb - 1) / v.wpb);
  return with_variant(v, phase, shuffle, [&](auto sc, auto wc, auto ic, auto pc, auto mc, auto hc) -> hipError_t {
    constexpr int S = decltype(sc)::value, W = decltype(wc)::value, PH = decltype(pc)::value;
    constexpr bool INC = decltype(ic)::value, MRT = decltype(mc)::value, SH = decltype(hc)::value;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * W), 0, s, src, dst, a, nrec, nrow, rbase, coef, list, count);
      return hipGetLastError();
    };
    auto by_mode = [&](auto nt) {
      constexpr bool NT = decltype(nt)::value;
      switch (mode) {
        case kDirect: return go(k_step19<S, W, NT, INC, PH, MRT, kDirect, SH>);
        case kList: return go(k_step19<S, W, NT, INC, PH, MRT, kList, SH>);
        default: return go(k_step19<S, W, NT, INC, PH, MRT, kPersistent, SH>);
      }
    };
    // MRT is built with non-temporal stores only (the planner rejects others)
    if constexpr (MRT) return by_mode(BC<true>{});
    else return nontemporal ? by_mode(BC<true>{}) : by_mode(BC<false>{});
  });
}

// Workgroups of the persistent step that fit on the device at once.
hipError_t step19_persistent_blocks(const Variant &v, bool single_copy, bool shuffle, int64_t *blocks) {
  int dev = 0, cus = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  // the grid must fit for every phase the solver alternates between
  auto fit = [&](int phase) -> hipError_t {
    return with_variant(v, phase, shuffle, [&](auto sc, auto wc, auto ic, auto pc, auto mc, auto hc) -> hipError_t {
      constexpr int S = decltype(sc)::value, W = decltype(wc)::value, PH = decltype(pc)::value;
      constexpr bool INC = decltype(ic)::value, MRT = decltype(mc)::value, SH = decltype(hc)::value;
      int k = 0;
      const hipError_t r = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &k, k_step19<S, W, true, INC, PH, MRT, kPersistent, SH>, 64 * W, 0);
      per = per < 0 ? k : (k < per ? k : per);
      return r;
    });
  };
  per = -1;
  if (e == hipSuccess) e = fit(single_copy ? kAAGather : kTwoCopy);
  if (e == hipSuccess && single_copy) e = fit(kAALocal);
  if (e != hipSuccess) return e;
  *blocks = (int64_t)cus * (per > 0 ? per : 1);
  return hipSuccess;
}

}  // namespace lbm
