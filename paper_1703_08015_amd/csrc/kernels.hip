// liblbm device kernels for gfx950 (CDNA4, wave64).
//
// Mapping: one 64-lane wavefront per 64 nodes of a tile (a 4x4x4 D3Q19 tile
// is exactly one wavefront; a 16x16 D2Q9 tile is four), lane l = node
// lx + ax*(ly + ay*lz) in the paper's row order (Sec. 3.2).  Solid lanes are
// masked off for the whole wavefront, so the PDF traffic is that of the
// non-solid nodes only.
//
// Storage: per non-empty tile, a region of q direction blocks holding only
// the tile's non-solid nodes, in lane order (rank r = number of non-solid
// lanes before the node).  A lane's own block-i entry is at off + i*n + r,
// so the 19 loads and stores of a tile's own nodes are contiguous runs.
//
// Step (gather form of the two-copy method, Sec. 3 and Fig. 5): each lane
// reads f_i from the node x - c_i, which may lie in one of the tile's
// neighbours (found through the neighbour row of the tile map); a solid or
// missing source means half-way bounce-back, f_i(x) = f*_opp(i)(x)
// (propagation only between non-solid nodes, Sec. 3.2).  Then the BGK
// collision of Eqs. (2) and (7) with Guo forcing, in the quasi-compressible
// model (Eqs. (3), (5)) or the incompressible one (Eqs. (4), (6)), and q stores.
// The neighbour records (region offset, node count, fluid bitmask) of the
// 3x3x3 tile neighbourhood are staged once per wavefront in LDS, as the
// paper stages the local tile bitmap and node types in shared memory.
//
// Single-copy form (one PDF buffer, steps in place; the addressing is
// described in step19.hip): the state after init or a local step holds f*_i
// in the node's slot opp(i); after a gather/scatter step it holds the
// streamed f_i in slot i, so f*_i(x) is then found where x + c_i reads it
// (slot i of x + c_i, or slot opp(i) of x when x + c_i is solid).  The
// auxiliary kernels read and write through that mapping.
#include "device.h"
#include "kernels.h"

namespace lbm {

template <int W>
struct Slot {
  int64_t off;
  uint64_t mask[W];
  int32_t n;
  int32_t pre[W];
};

// Stage the neighbour records of `tile` into LDS (lanes 0..26, one each).
template <class L, int W>
__device__ __forceinline__ void stage_slots(Slot<W> *slots, const TileArgs &a, int64_t tile, int lane) {
  if (lane >= 27) return;
  const int dx = lane % 3 - 1, dy = (lane / 3) % 3 - 1, dz = lane / 9 - 1;
  const int reach = (dx != 0) + (dy != 0) + (dz != 0);
  // D2Q9 never leaves the z = 0 plane; D3Q19 has no corner directions
  const bool need = (L::Q == 9) ? (dz == 0 && reach <= 2) : (reach <= 2);
  const int32_t t2 = need ? a.nbr[tile * 27 + lane] : -1;
  Slot<W> s;
  if (t2 >= 0) {
    const TileRec r = a.rec[t2];
    s.off = r.off;
    s.n = r.n;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      s.mask[w] = a.fluid[(int64_t)t2 * W + w];
      s.pre[w] = (W == 1) ? 0 : a.pre[(int64_t)t2 * W + w];
    }
  } else {
    s.off = 0;
    s.n = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      s.mask[w] = 0ull;
      s.pre[w] = 0;
    }
  }
  slots[lane] = s;
}

__device__ __forceinline__ int lane_rank(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// ---- fused step -----------------------------------------------------------------
// The two-copy D2Q9 BGK step asks for 8 waves per SIMD: left to itself the
// compiler clusters the loads of a 16x16 tile into 76 VGPRs (6 waves), where
// 56 registers with no extra instructions give all 8 (+5% measured; the
// single-copy phases measured slower with 8 and keep the compiler's choice)
template <class L, int AX, int AY, int AZ, int S, int WPB, bool INC, int PH, bool MRT>
__global__ void __launch_bounds__(64 * WPB)
    __attribute__((amdgpu_waves_per_eu(L::Q == 9 && !MRT && PH == kPhaseTwoCopy ? 8 : 1)))
    k_step(in_ptr<PH, void> src_, out_ptr<PH, void> dst_, TileArgs a, double omega_d) {
  using St = Store<S>;
  using T = typename St::T;
  using R = typename St::R;
  constexpr int Q = L::Q;
  constexpr int W = AX * AY * AZ / 64;
  __shared__ Slot<W> slots[WPB][27];
  in_ptr<PH, T> src = static_cast<const T *>(src_);
  out_ptr<PH, T> dst = static_cast<T *>(dst_);

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // D2Q9 hands the XCDs chunks of 8 workgroups in turn (+2.5% FP64, +6% FP32
  // measured on the 4096^2 channel against one contiguous range per XCD)
  const int64_t blk = L::Q == 9 ? xcd_chunk(blockIdx.x, gridDim.x, 8) : xcd_remap(blockIdx.x, gridDim.x);
  const int64_t gw = blk * WPB + wv;
  const bool valid = gw < a.n_waves;
  const int64_t tile = gw / W;
  const int part = (int)(gw % W);
  if (valid) stage_slots<L, W>(slots[wv], a, tile, lane);
  __syncthreads();
  if (!valid) return;

  const Slot<W> &own = slots[wv][13];
  const uint64_t M = own.mask[part];
  if (!((M >> lane) & 1ull)) return;
  const int ell = part * 64 + lane;
  const int x = ell % AX, y = (ell / AX) % AY, z = ell / (AX * AY);
  const int rank = own.pre[part] + lane_rank(M);
  const int64_t obase = own.off + rank;
  const int on = own.n;

  R f[Q];
  int64_t ea[PH == kPhaseAAGather ? Q : 1];  // entries read, rewritten by the single-copy gather
  static_for<Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = L::C[i][0], cy = L::C[i][1], cz = L::C[i][2];
    constexpr int ib = PH == kPhaseAAGather ? L::Opp[i] : i;  // slot of the source's value
    int64_t addr;
    if constexpr (i == 0 || PH == kPhaseAALocal) {
      addr = obase + (int64_t)i * on;
    } else {
      int sx = x - cx, sy = y - cy, sz = z - cz, dx = 0, dy = 0, dz = 0;
      if constexpr (cx != 0) {
        if (sx < 0) { dx = -1; sx += AX; } else if (sx >= AX) { dx = 1; sx -= AX; }
      }
      if constexpr (cy != 0) {
        if (sy < 0) { dy = -1; sy += AY; } else if (sy >= AY) { dy = 1; sy -= AY; }
      }
      if constexpr (cz != 0) {
        if (sz < 0) { dz = -1; sz += AZ; } else if (sz >= AZ) { dz = 1; sz -= AZ; }
      }
      const Slot<W> &sl = slots[wv][13 + dx + 3 * dy + 9 * dz];
      const int s = sx + AX * (sy + AY * sz);
      const int wd = (W == 1) ? 0 : (s >> 6);
      const int b = s & 63;
      const uint64_t m = sl.mask[wd];
      if ((m >> b) & 1ull)
        addr = sl.off + (int64_t)ib * sl.n + sl.pre[wd] + __popcll(m & ((1ull << b) - 1ull));
      else  // half-way bounce-back: the node's own value opp(i), in slot opp(i) (slot i in place)
        addr = obase + (int64_t)(PH == kPhaseAAGather ? i : L::Opp[i]) * on;
    }
    f[i] = St::load(src, addr, a.f16_inv);
    if constexpr (PH == kPhaseAAGather) ea[i] = addr;
  });
  // macroscopic moments, Eq. (5) or (6) with the half-force shift
  const SampleRec &smp = a.samples[a.rec[tile].sample];
  const R gx = (R)smp.g[0], gy = (R)smp.g[1], gz = (R)smp.g[2];
  R sum = 0, jx = 0, jy = 0, jz = 0;
  static_for<Q>([&](auto I) {
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
  const R rho = St::offset ? (R)a.rho0 + sum : sum;
  const R m = velocity_density<INC>(rho);
  R ux, uy, uz;
  if constexpr (INC) {
    ux = jx + R(0.5) * gx, uy = jy + R(0.5) * gy, uz = jz + R(0.5) * gz;
  } else {
    const R inv = R(1) / rho;
    ux = jx * inv + R(0.5) * gx, uy = jy * inv + R(0.5) * gy, uz = jz * inv + R(0.5) * gz;
  }
  const R uu = ux * ux + uy * uy + uz * uz;
  const R om = (R)omega_d;
  const R fo = R(1) - R(0.5) * om;

  // two-copy: own slot i; single-copy gather: where opp(i) was read;
  // single-copy local: own slot opp(i)
  auto put = [&](auto I, R out) {
    constexpr int i = decltype(I)::value;
    int64_t e;
    if constexpr (PH == kPhaseTwoCopy)
      e = obase + (int64_t)i * on;
    else if constexpr (PH == kPhaseAAGather)
      e = ea[L::Opp[i]];
    else
      e = obase + (int64_t)L::Opp[i] * on;
    St::store(dst, e, out, a.f16_scale);
  };
  if constexpr (MRT) {
    // Eq. (8) in the orthogonal moment basis
    collide_mrt<L, S, INC>(f, sum, jx, jy, jz, (R)a.rho0, gx, gy, gz, a.mrt);
    static_for<Q>([&](auto I) { put(I, f[decltype(I)::value]); });
    return;
  }
  // BGK collision, Eqs. (2), (3) or (4), (7) + Guo source; store own block entries
  static_for<Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = L::C[i][0], cy = L::C[i][1], cz = L::C[i][2];
    constexpr R w = (R)L::Wt[i];
    const R cu = R(cx) * ux + R(cy) * uy + R(cz) * uz;
    const R cg = R(cx) * gx + R(cy) * gy + R(cz) * gz;
    const R cmug = (R(cx) - ux) * gx + (R(cy) - uy) * gy + (R(cz) - uz) * gz;
    const R poly = R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;
    // full form: w (rho + m poly); offset form: w (drho + m poly), m = rho or 1
    R feq;
    if constexpr (INC) feq = St::offset ? w * (sum + poly) : w * (rho + poly);
    else feq = St::offset ? w * (sum + rho * poly) : w * rho * (R(1) + poly);
    const R F = w * m * (R(3) * cmug + R(9) * cu * cg);
    put(I, f[i] + om * (feq - f[i]) + fo * F);
  });
}

// ---- per-node helpers for the auxiliary kernels -------------------------------
template <int AX, int AY, int AZ>
struct NodeCtx {
  bool fluid;
  int64_t tile;   // internal tile index
  int ell;        // node index inside the tile
  int64_t entry;  // own direction-0 entry
  int n;          // own tile's fluid count
  int64_t node;   // compact fluid-node index
  int64_t loc;    // index inside the sample's dense lattice
  int sample;
};

template <int AX, int AY, int AZ>
__device__ __forceinline__ NodeCtx<AX, AY, AZ> node_ctx(const TileArgs &a, int64_t gw) {
  constexpr int W = AX * AY * AZ / 64;
  NodeCtx<AX, AY, AZ> c;
  const int lane = threadIdx.x & 63;
  const int64_t tile = gw / W;
  const int part = (int)(gw % W);
  const uint64_t M = a.fluid[tile * W + part];
  c.fluid = (M >> lane) & 1ull;
  const int pre = (W == 1) ? 0 : a.pre[tile * W + part];
  const int rank = pre + lane_rank(M);
  c.tile = tile;
  c.ell = part * 64 + lane;
  const TileRec r = a.rec[tile];
  c.entry = r.off + rank;
  c.n = r.n;
  c.sample = r.sample;
  c.node = a.nbase[tile] + rank;
  const int ell = part * 64 + lane;
  const int x = ell % AX, y = (ell / AX) % AY, z = ell / (AX * AY);
  const SampleRec &s = a.samples[r.sample];
  const int64_t X = (int64_t)a.coord[3 * tile] * AX + x;
  const int64_t Y = (int64_t)a.coord[3 * tile + 1] * AY + y;
  const int64_t Z = (int64_t)a.coord[3 * tile + 2] * AZ + z;
  c.loc = X + s.shape[0] * (Y + (int64_t)s.shape[1] * Z);
  return c;
}

// Layout of the stored state of a node: -1 two-copy (f*_i in slot i); for the
// single copy 0 (f*_i in slot opp(i), after init, import or a local step) or
// 1 (streamed values, after a gather/scatter step).  A sample taken out of
// the active list stays at layout 0 (the solver only freezes it there).
template <int AX, int AY, int AZ>
__device__ __forceinline__ int node_layout(const TileArgs &a, const NodeCtx<AX, AY, AZ> &c) {
  if (a.aa_phase < 0) return -1;
  return a.samples[c.sample].frozen ? 0 : a.aa_phase;
}

// Entry that holds the post-collision value f*_i of the node.
template <class L, int AX, int AY, int AZ, int i>
__device__ __forceinline__ int64_t post_entry(const TileArgs &a, const NodeCtx<AX, AY, AZ> &c, int layout) {
  constexpr int W = AX * AY * AZ / 64;
  if (layout < 0) return c.entry + (int64_t)i * c.n;
  if (layout == 1 && i != 0) {
    // f*_i(x) is what x + c_i pulls next: slot i of x + c_i when that node is fluid
    int x = c.ell % AX + L::C[i][0], y = (c.ell / AX) % AY + L::C[i][1], z = c.ell / (AX * AY) + L::C[i][2];
    int dx = 0, dy = 0, dz = 0;
    if (x < 0) { dx = -1; x += AX; } else if (x >= AX) { dx = 1; x -= AX; }
    if (y < 0) { dy = -1; y += AY; } else if (y >= AY) { dy = 1; y -= AY; }
    if (z < 0) { dz = -1; z += AZ; } else if (z >= AZ) { dz = 1; z -= AZ; }
    const int64_t t2 = (dx | dy | dz) ? (int64_t)a.nbr[c.tile * 27 + 13 + dx + 3 * dy + 9 * dz] : c.tile;
    if (t2 >= 0) {
      const int s = x + AX * (y + AY * z), wd = (W == 1) ? 0 : (s >> 6), b = s & 63;
      const uint64_t m = a.fluid[t2 * W + wd];
      if ((m >> b) & 1ull) {
        const TileRec r = a.rec[t2];
        const int pre = (W == 1) ? 0 : a.pre[t2 * W + wd];
        return r.off + (int64_t)i * r.n + pre + __popcll(m & ((1ull << b) - 1ull));
      }
    }
  }
  // slot opp(i) of the node itself (layout 0, or bounced back in layout 1)
  return c.entry + (int64_t)L::Opp[i] * c.n;
}

// Entry to write f*_i of the node when setting a state (init, import): the
// layout the next step expects.
template <class L, int AX, int AY, int AZ, int i>
__device__ __forceinline__ int64_t set_entry(const TileArgs &a, const NodeCtx<AX, AY, AZ> &c) {
  return c.entry + (int64_t)(a.aa_phase < 0 ? i : L::Opp[i]) * c.n;
}

// FP64 value of stored PDF i of a node.
template <class L, int S, int i>
__device__ __forceinline__ double load_f64(const void *src, int64_t e, const TileArgs &a) {
  using St = Store<S>;
  const double v = (double)St::load(static_cast<const typename St::T *>(src), e, a.f16_inv);
  return St::offset ? L::Wt[i] * a.rho0 + v : v;
}

// rho = sum f*, j = sum c f* (FP64, from the stored state).  For offsets,
// rho = rho0 + sum of offsets (the weights sum to one, the first moment of
// w_i rho0 vanishes).
template <class L, int S, int AX, int AY, int AZ>
__device__ __forceinline__ void stored_moments(const void *src, const NodeCtx<AX, AY, AZ> &c, const TileArgs &a,
                                               double &rho, double (&j)[3]) {
  using St = Store<S>;
  const int layout = node_layout(a, c);
  double sum = 0.0;
  j[0] = j[1] = j[2] = 0.0;
  static_for<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    const int64_t e = post_entry<L, AX, AY, AZ, i>(a, c, layout);
    const double v = (double)St::load(static_cast<const typename St::T *>(src), e, a.f16_inv);
    sum += v;
    j[0] += L::C[i][0] * v;
    j[1] += L::C[i][1] * v;
    j[2] += L::C[i][2] * v;
  });
  rho = St::offset ? a.rho0 + sum : sum;
}

template <class L, int AX, int AY, int AZ, int S>
__global__ void __launch_bounds__(256) k_init(void *dst_, TileArgs a, const double *rho, const double *u) {
  using St = Store<S>;
  const int64_t gw = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (gw >= a.n_waves) return;
  const NodeCtx<AX, AY, AZ> c = node_ctx<AX, AY, AZ>(a, gw);
  if (!c.fluid) return;
  const SampleRec &s = a.samples[c.sample];
  const double r = rho ? rho[s.dense0 + c.loc] : a.rho0;
  double v[3] = {0.0, 0.0, 0.0};
  if (u)
    for (int k = 0; k < 3; ++k) v[k] = u[3 * s.dense0 + k * s.n_nodes + c.loc];
  const double uu = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const bool inc = a.model == LBM_MODEL_INCOMPRESSIBLE;
  typename St::T *dst = static_cast<typename St::T *>(dst_);
  static_for<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    const double cu = L::C[i][0] * v[0] + L::C[i][1] * v[1] + L::C[i][2] * v[2];
    const double poly = 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
    // Eq. (4) or Eq. (3)
    const double fe = inc ? L::Wt[i] * (r + poly) : L::Wt[i] * r * (1.0 + poly);
    const double val = St::offset ? fe - L::Wt[i] * a.rho0 : fe;
    St::store(dst, set_entry<L, AX, AY, AZ, i>(a, c), (typename St::R)val, a.f16_scale);
  });
}

template <class L, int AX, int AY, int AZ, int S>
__global__ void __launch_bounds__(256) k_moments(const void *src, TileArgs a, double *rho, double *u) {
  const int64_t gw = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (gw >= a.n_waves) return;
  const NodeCtx<AX, AY, AZ> c = node_ctx<AX, AY, AZ>(a, gw);
  if (!c.fluid) return;
  const SampleRec &s = a.samples[c.sample];
  double r, j[3];
  stored_moments<L, S>(src, c, a, r, j);
  if (rho) rho[s.dense0 + c.loc] = r;
  const double m = a.model == LBM_MODEL_INCOMPRESSIBLE ? 1.0 : r;
  if (u)
    for (int k = 0; k < 3; ++k) u[3 * s.dense0 + k * s.n_nodes + c.loc] = j[k] / m - 0.5 * s.g[k];
}

template <class L, int AX, int AY, int AZ, int S>
__global__ void __launch_bounds__(256) k_export(const void *src, TileArgs a, double *dense) {
  const int64_t gw = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (gw >= a.n_waves) return;
  const NodeCtx<AX, AY, AZ> c = node_ctx<AX, AY, AZ>(a, gw);
  if (!c.fluid) return;
  const SampleRec &s = a.samples[c.sample];
  const int layout = node_layout(a, c);
  static_for<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    dense[L::Q * s.dense0 + i * s.n_nodes + c.loc] = load_f64<L, S, i>(src, post_entry<L, AX, AY, AZ, i>(a, c, layout), a);
  });
}

template <class L, int AX, int AY, int AZ, int S>
__global__ void __launch_bounds__(256) k_import(void *dst_, TileArgs a, const double *dense) {
  using St = Store<S>;
  const int64_t gw = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (gw >= a.n_waves) return;
  const NodeCtx<AX, AY, AZ> c = node_ctx<AX, AY, AZ>(a, gw);
  if (!c.fluid) return;
  const SampleRec &s = a.samples[c.sample];
  typename St::T *dst = static_cast<typename St::T *>(dst_);
  static_for<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    const double v = dense[L::Q * s.dense0 + i * s.n_nodes + c.loc];
    const double val = St::offset ? v - L::Wt[i] * a.rho0 : v;
    St::store(dst, set_entry<L, AX, AY, AZ, i>(a, c), (typename St::R)val, a.f16_scale);
  });
}

// Moving wall (the lid of a driven cavity).  The value that a lid node x
// pulls next step for a direction i from beyond the lid face is its own
// bounce-back value f*_opp(i)(x), and no other node reads that entry; so the
// wall's term corr_i = 6 w_i rho_w (c_i . u_w) is added to it just before the
// step, and the step's gather sees exactly f*_opp(i)(x) + corr_i.  The entry
// is slot opp(i) of the node in the two-copy source, slot i in either layout
// of the single copy.  One wavefront per 64 nodes of a listed tile (the
// tiles holding the lattice's first or last row along the lid's axis).
template <class L, int AX, int AY, int AZ, int S>
__global__ void __launch_bounds__(256)
    k_lid_fixup(void *buf_, TileArgs a, const int32_t *__restrict__ tiles, int64_t n_waves, int own_slot) {
  using St = Store<S>;
  using R = typename St::R;
  constexpr int W = AX * AY * AZ / 64;
  const int64_t gw = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (gw >= n_waves) return;
  const NodeCtx<AX, AY, AZ> c = node_ctx<AX, AY, AZ>(a, (int64_t)tiles[gw / W] * W + gw % W);
  if (!c.fluid || a.samples[c.sample].frozen) return;  // a frozen sample keeps its state
  const int ax = a.lid.axis;
  const int x = c.ell % AX, y = (c.ell / AX) % AY, z = c.ell / (AX * AY);
  const int p = a.coord[3 * c.tile + ax] * (ax == 0 ? AX : ax == 1 ? AY : AZ) + (ax == 0 ? x : ax == 1 ? y : z);
  const int n = a.samples[c.sample].shape[ax];
  if (p != (a.lid.side ? n - 1 : 0)) return;
  const int toward = a.lid.side ? -1 : 1;  // c along the axis of a pull from beyond the face
  typename St::T *buf = static_cast<typename St::T *>(buf_);
  static_for<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    const int ca = ax == 0 ? L::C[i][0] : ax == 1 ? L::C[i][1] : L::C[i][2];
    if (ca != toward) return;
    const int64_t e = c.entry + (int64_t)(own_slot ? i : L::Opp[i]) * c.n;
    const R v = St::load(buf, e, a.f16_inv) + (St::offset ? (R)a.lid.corrf[i] : (R)a.lid.corr[i]);
    St::store(buf, e, v, a.f16_scale);
  });
}

// Fixed-order wavefront sum (butterfly); every lane ends with the total.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <class L, int AX, int AY, int AZ, int S>
__global__ void __launch_bounds__(256) k_reduce_partial(const void *src, TileArgs a, double *part) {
  const int64_t gw = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (gw >= a.n_waves) return;  // uniform per wavefront
  const NodeCtx<AX, AY, AZ> c = node_ctx<AX, AY, AZ>(a, gw);
  double m = 0.0, p[3] = {0.0, 0.0, 0.0};
  if (c.fluid) {
    const SampleRec &s = a.samples[c.sample];
    double j[3];
    stored_moments<L, S>(src, c, a, m, j);
    // rho u, or u at the incompressible model's reference density 1
    const double d = a.model == LBM_MODEL_INCOMPRESSIBLE ? 1.0 : m;
    for (int k = 0; k < 3; ++k) p[k] = j[k] - 0.5 * d * s.g[k];
  }
  m = wave_sum(m);
  for (int k = 0; k < 3; ++k) p[k] = wave_sum(p[k]);
  if ((threadIdx.x & 63) == 0) {
    part[4 * gw] = m;
    for (int k = 0; k < 3; ++k) part[4 * gw + 1 + k] = p[k];
  }
}

template <class L, int AX, int AY, int AZ, int S>
__global__ void __launch_bounds__(256)
    k_residual_partial(const void *src, TileArgs a, double *uref, double *part, int accumulate) {
  const int64_t gw = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (gw >= a.n_waves) return;
  const NodeCtx<AX, AY, AZ> c = node_ctx<AX, AY, AZ>(a, gw);
  double d2 = 0.0, n2 = 0.0;
  if (c.fluid) {
    const SampleRec &s = a.samples[c.sample];
    double r, j[3];
    stored_moments<L, S>(src, c, a, r, j);
    const double m = a.model == LBM_MODEL_INCOMPRESSIBLE ? 1.0 : r;
    for (int k = 0; k < 3; ++k) {
      const double uk = j[k] / m - 0.5 * s.g[k];
      double *ref = uref + (int64_t)k * a.n_fluid + c.node;
      const double dk = uk - *ref;
      d2 += dk * dk;
      n2 += uk * uk;
      *ref = uk;
    }
  }
  if (!accumulate) return;
  d2 = wave_sum(d2);
  n2 = wave_sum(n2);
  if ((threadIdx.x & 63) == 0) {
    part[2 * gw] = d2;
    part[2 * gw + 1] = n2;
  }
}

// Fixed-order sum of per-wave partials, in two stages.  Stage 1: block
// (c, s) sums chunk c of sample s's waves -- thread t takes partials t,
// t+256, ... of the chunk in order, then a fixed shared-memory tree.  Stage 2:
// one 64-thread block per sample sums the kReduceChunks chunk totals with a
// fixed tree.  The launch shape is fixed, so results repeat bit for bit.
constexpr int kReduceChunks = 64;

__global__ void __launch_bounds__(256)
    k_reduce_chunks(const double *part, int ncomp, const SampleRec *samples, int words, double *chunk_out) {
  __shared__ double sh[256 * 4];
  const SampleRec &s = samples[blockIdx.y];
  const int64_t w0 = s.tile0 * words, n = s.n_ftiles * words;
  const int64_t per = (n + kReduceChunks - 1) / kReduceChunks;
  const int64_t c0 = w0 + per * blockIdx.x;
  const int64_t c1 = (c0 + per < w0 + n) ? c0 + per : w0 + n;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t w = c0 + threadIdx.x; w < c1; w += 256)
    for (int k = 0; k < ncomp; ++k) acc[k] += part[ncomp * w + k];
  for (int k = 0; k < ncomp; ++k) sh[k * 256 + threadIdx.x] = acc[k];
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int k = 0; k < ncomp; ++k) sh[k * 256 + threadIdx.x] += sh[k * 256 + threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < (unsigned)ncomp)
    chunk_out[((int64_t)blockIdx.y * kReduceChunks + blockIdx.x) * ncomp + threadIdx.x] = sh[threadIdx.x * 256];
}

__global__ void __launch_bounds__(64) k_reduce_final(const double *chunk, int ncomp, double *out) {
  __shared__ double sh[64 * 4];
  for (int k = 0; k < ncomp; ++k)
    sh[k * 64 + threadIdx.x] = chunk[((int64_t)blockIdx.x * kReduceChunks + threadIdx.x) * ncomp + k];
  __syncthreads();
  for (int o = 32; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int k = 0; k < ncomp; ++k) sh[k * 64 + threadIdx.x] += sh[k * 64 + threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < (unsigned)ncomp) out[ncomp * blockIdx.x + threadIdx.x] = sh[threadIdx.x * 64];
}

__global__ void k_fill(double *p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---- dispatch -------------------------------------------------------------------
int storage_bytes(int storage) {
  return storage == LBM_F64 ? 8 : storage == LBM_F32_OFFSET ? 4 : storage == LBM_F16_OFFSET ? 2 : 0;
}

bool variant_supported(const Variant &v) {
  if (storage_bytes(v.storage) == 0) return false;
  if (v.model != LBM_MODEL_QUASI_COMPRESSIBLE && v.model != LBM_MODEL_INCOMPRESSIBLE) return false;
  if (v.collision != LBM_COLLISION_BGK && v.collision != LBM_COLLISION_MRT) return false;
  if (v.q == 9) return v.ax == 16 && v.ay == 16 && v.az == 1 && v.wpb == 4;
  if (v.q == 19)
    return v.ax == 4 && v.ay == 4 && (v.az == 4 || v.az == 8) &&
           (v.wpb == 1 || v.wpb == 2 || v.wpb == 4 || v.wpb == 8);
  return false;
}

// Calls f.template operator()<L, AX, AY, AZ, S, WPB>() for the variant.
template <class F>
static hipError_t dispatch(const Variant &v, F &&f) {
  if (!variant_supported(v)) return hipErrorInvalidValue;
  auto by_storage = [&](auto lat, auto ax, auto ay, auto az, auto wpb) -> hipError_t {
    using L = decltype(lat);
    constexpr int AX = decltype(ax)::value, AY = decltype(ay)::value, AZ = decltype(az)::value;
    constexpr int WPB = decltype(wpb)::value;
    switch (v.storage) {
      case LBM_F64: return f.template operator()<L, AX, AY, AZ, LBM_F64, WPB>();
      case LBM_F32_OFFSET: return f.template operator()<L, AX, AY, AZ, LBM_F32_OFFSET, WPB>();
      default: return f.template operator()<L, AX, AY, AZ, LBM_F16_OFFSET, WPB>();
    }
  };
  using I4 = std::integral_constant<int, 4>;
  using I8 = std::integral_constant<int, 8>;
  using I16 = std::integral_constant<int, 16>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  if (v.q == 9) return by_storage(D2Q9{}, I16{}, I16{}, I1{}, I4{});
  auto by_wpb = [&](auto az) -> hipError_t {
    switch (v.wpb) {
      case 1: return by_storage(D3Q19{}, I4{}, I4{}, az, I1{});
      case 2: return by_storage(D3Q19{}, I4{}, I4{}, az, I2{});
      case 4: return by_storage(D3Q19{}, I4{}, I4{}, az, I4{});
      default: return by_storage(D3Q19{}, I4{}, I4{}, az, I8{});
    }
  };
  return v.az == 4 ? by_wpb(I4{}) : by_wpb(I8{});
}

static unsigned blocks_for(int64_t waves, int per_block) { return (unsigned)((waves + per_block - 1) / per_block); }

hipError_t launch_step(const Variant &v, int phase, const void *src, void *dst, const TileArgs &a, double omega,
                       hipStream_t s) {
  if (a.n_waves == 0) return hipSuccess;
  if ((phase == kPhaseTwoCopy) == (src == dst)) return hipErrorInvalidValue;  // in place exactly for the single copy
  return dispatch(v, [&]<class L, int AX, int AY, int AZ, int S, int WPB>() {
    auto go = [&](auto inc, auto ph) {
      constexpr bool INC = decltype(inc)::value;
      constexpr int PH = decltype(ph)::value;
      // MRT is built for 4 waves per workgroup only (the planner rejects others)
      if constexpr (WPB == 4)
        if (v.collision == LBM_COLLISION_MRT) {
          hipLaunchKernelGGL((k_step<L, AX, AY, AZ, S, WPB, INC, PH, true>), dim3(blocks_for(a.n_waves, WPB)),
                             dim3(64 * WPB), 0, s, src, dst, a, omega);
          return;
        }
        hipLaunchKernelGGL((k_step<L, AX, AY, AZ, S, WPB, INC, PH, false>), dim3(blocks_for(a.n_waves, WPB)),
                           dim3(64 * WPB), 0, s, src, dst, a, omega);
    };
    auto by_phase = [&](auto inc) {
      switch (phase) {
        case kPhaseAAGather: go(inc, std::integral_constant<int, kPhaseAAGather>{}); break;
        case kPhaseAALocal: go(inc, std::integral_constant<int, kPhaseAALocal>{}); break;
        default: go(inc, std::integral_constant<int, kPhaseTwoCopy>{});
      }
    };
    if (v.model == LBM_MODEL_INCOMPRESSIBLE)
      by_phase(std::true_type{});
    else
      by_phase(std::false_type{});
    return hipGetLastError();
  });
}

// The auxiliary kernels do not depend on the workgroup size of the step.
static Variant aux(const Variant &v) {
  Variant w = v;
  if (w.q == 19) w.wpb = 4;
  return w;
}

hipError_t launch_init(const Variant &v, void *dst, const TileArgs &a, const double *rho, const double *u,
                       hipStream_t s) {
  if (a.n_waves == 0) return hipSuccess;
  return dispatch(aux(v), [&]<class L, int AX, int AY, int AZ, int S, int WPB>() {
    hipLaunchKernelGGL((k_init<L, AX, AY, AZ, S>), dim3(blocks_for(a.n_waves, 4)), dim3(256), 0, s, dst, a, rho, u);
    return hipGetLastError();
  });
}

hipError_t launch_moments(const Variant &v, const void *src, const TileArgs &a, double *rho, double *u,
                          hipStream_t s) {
  if (a.n_waves == 0) return hipSuccess;
  return dispatch(aux(v), [&]<class L, int AX, int AY, int AZ, int S, int WPB>() {
    hipLaunchKernelGGL((k_moments<L, AX, AY, AZ, S>), dim3(blocks_for(a.n_waves, 4)), dim3(256), 0, s, src, a, rho,
                       u);
    return hipGetLastError();
  });
}

hipError_t launch_export(const Variant &v, const void *src, const TileArgs &a, double *dense, hipStream_t s) {
  if (a.n_waves == 0) return hipSuccess;
  return dispatch(aux(v), [&]<class L, int AX, int AY, int AZ, int S, int WPB>() {
    hipLaunchKernelGGL((k_export<L, AX, AY, AZ, S>), dim3(blocks_for(a.n_waves, 4)), dim3(256), 0, s, src, a, dense);
    return hipGetLastError();
  });
}

hipError_t launch_import(const Variant &v, void *dst, const TileArgs &a, const double *dense, hipStream_t s) {
  if (a.n_waves == 0) return hipSuccess;
  return dispatch(aux(v), [&]<class L, int AX, int AY, int AZ, int S, int WPB>() {
    hipLaunchKernelGGL((k_import<L, AX, AY, AZ, S>), dim3(blocks_for(a.n_waves, 4)), dim3(256), 0, s, dst, a, dense);
    return hipGetLastError();
  });
}

hipError_t launch_reduce_partial(const Variant &v, const void *src, const TileArgs &a, double *part,
                                 hipStream_t s) {
  if (a.n_waves == 0) return hipSuccess;
  return dispatch(aux(v), [&]<class L, int AX, int AY, int AZ, int S, int WPB>() {
    hipLaunchKernelGGL((k_reduce_partial<L, AX, AY, AZ, S>), dim3(blocks_for(a.n_waves, 4)), dim3(256), 0, s, src,
                       a, part);
    return hipGetLastError();
  });
}

hipError_t launch_residual_partial(const Variant &v, const void *src, const TileArgs &a, double *uref,
                                   double *part, int accumulate, hipStream_t s) {
  if (a.n_waves == 0) return hipSuccess;
  return dispatch(aux(v), [&]<class L, int AX, int AY, int AZ, int S, int WPB>() {
    hipLaunchKernelGGL((k_residual_partial<L, AX, AY, AZ, S>), dim3(blocks_for(a.n_waves, 4)), dim3(256), 0, s,
                       src, a, uref, part, accumulate);
    return hipGetLastError();
  });
}

hipError_t launch_lid_fixup(const Variant &v, void *buf, const TileArgs &a, const int32_t *tiles, int64_t n_tiles,
                            int own_slot, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  const int64_t waves = n_tiles * (v.ax * v.ay * v.az / 64);
  return dispatch(aux(v), [&]<class L, int AX, int AY, int AZ, int S, int WPB>() {
    hipLaunchKernelGGL((k_lid_fixup<L, AX, AY, AZ, S>), dim3(blocks_for(waves, 4)), dim3(256), 0, s, buf, a, tiles,
                       waves, own_slot);
    return hipGetLastError();
  });
}

int reduce_chunks() { return kReduceChunks; }

hipError_t launch_reduce_final(const double *part, int ncomp, const SampleRec *samples, int n_samples, int words,
                               double *chunk, double *out, hipStream_t s) {
  if (n_samples <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_chunks, dim3(kReduceChunks, n_samples), dim3(256), 0, s, part, ncomp, samples, words,
                     chunk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final, dim3(n_samples), dim3(64), 0, s, chunk, ncomp, out);
  return hipGetLastError();
}

hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace lbm
