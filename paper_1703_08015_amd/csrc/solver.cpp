// Solver runtime behind the C ABI of lbm.h: validates parameters, lays out
// the caller's device workspace (two PDF copies of the two-copy method,
// Sec. 3, tile tables and reduction scratch), uploads the tiling and
// enqueues the kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "device.h"
#include "internal.h"
#include "kernels.h"

using lbm::set_error;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Byte offsets of every workspace array, plus the host tables to upload.
struct Plan {
  size_t buf[2], rec, fluid, pre, nbr, coord, nbase, samples, coef, nrec, nrow, rbase, list, lid, count, part, chunk, out,
      uref, total;
  int64_t entries = 0;  // PDF entries per copy (with region alignment padding)
  // device tables in the solver's internal tile order
  std::vector<lbm::TileRec> rec_h;
  std::vector<uint64_t> fluid_h;
  std::vector<int32_t> pre_h, nbr_h, coord_h;
  std::vector<int64_t> nbase_h;
  std::vector<lbm::SampleRec> samples_h;
  std::vector<lbm::CollideCoef> coef_h;
  // scalar-mask D3Q19 kernel: compact records (+ all-solid sentinel) and rows
  std::vector<lbm::NbRec> nrec_h;
  std::vector<uint32_t> nrow_h;   // byte offsets into nrec
  std::vector<uint32_t> rbase_h;  // kRegionBases per tile: base entry of each lane region
};

// Neighbour slots (3x3x3 index) of the D3Q19 gather, in the order the
// scalar-mask kernel reads its compact neighbour row.
constexpr int kGatherSlots[18] = {4, 22, 10, 16, 12, 14, 1, 3, 5, 7, 9, 11, 15, 17, 19, 21, 23, 25};

// Morton (Z-order) key of a tile coordinate.
uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  auto spread = [](uint64_t v) {
    v &= 0x1fffffull;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
  };
  return spread(x) | spread(y) << 1 | spread(z) << 2;
}

void fill_coef(lbm::CollideCoef &c, const double g[3], double omega) {
  const double fo = 1.0 - 0.5 * omega;
  for (int a = 0; a < 3; ++a) c.g[a] = g[a];
  c.omega = omega;
  for (int i = 0; i < 19; ++i) {
    const double cg = lbm::D3Q19::C[i][0] * g[0] + lbm::D3Q19::C[i][1] * g[1] + lbm::D3Q19::C[i][2] * g[2];
    c.a[i] = 3.0 * omega + 9.0 * fo * cg;
    c.b[i] = 3.0 * fo * cg;
    c.af[i] = (float)c.a[i];
    c.bf[i] = (float)c.b[i];
  }
}

// Per-class terms of the MRT collision: -s and 1 - s/2, with s = omega for the
// shear stress, 1 for the conserved moments, the given rates (or the
// published defaults of the lattice) for the others.
lbm::MrtRates mrt_rates(const lbm_params *p, double omega) {
  static const double d19[5] = {1.19, 1.4, 1.2, 1.4, 1.98}, d9[5] = {1.64, 1.54, 1.9, 1.0, 1.0};
  const double *def = p->lattice == 9 ? d9 : d19;
  double s[lbm::kMrtClasses];
  s[lbm::kMrtCons] = 1.0;
  s[lbm::kMrtNu] = omega;
  const int cls[5] = {lbm::kMrtE, lbm::kMrtEps, lbm::kMrtQ, lbm::kMrtPi, lbm::kMrtM};
  for (int k = 0; k < 5; ++k) s[cls[k]] = p->mrt_rates[k] != 0.0 ? p->mrt_rates[k] : def[k];
  lbm::MrtRates r;
  for (int c = 0; c < lbm::kMrtClasses; ++c) {
    r.ms[c] = -s[c];
    r.mh[c] = 1.0 - 0.5 * s[c];
    r.msf[c] = (float)r.ms[c];
    r.mhf[c] = (float)r.mh[c];
  }
  return r;
}

int check_params(const lbm_tiles *t, const lbm_params *p, lbm::Variant *v) {
  if (!t || !p) return set_error(LBM_ERR_ARG, "NULL tiles or params");
  if (lbm::storage_bytes(p->storage) == 0) return set_error(LBM_ERR_ARG, "unknown storage form %d", p->storage);
  const bool tau_inf = std::isinf(p->tau) && p->tau > 0;
  if (!tau_inf && !(std::isfinite(p->tau) && p->tau > 0.5))
    return set_error(LBM_ERR_ARG, "tau = %g: must exceed 1/2 (or be +inf)", p->tau);
  if (!(std::isfinite(p->rho0) && p->rho0 > 0)) return set_error(LBM_ERR_ARG, "rho0 = %g", p->rho0);
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->g[a])) return set_error(LBM_ERR_ARG, "g[%d] is not finite", a);
  if (p->f16_scale_log2 < 0 || p->f16_scale_log2 > 24)
    return set_error(LBM_ERR_ARG, "f16_scale_log2 = %d outside 0..24", p->f16_scale_log2);
  if (p->tile_order != LBM_ORDER_MORTON && p->tile_order != LBM_ORDER_ROWMAJOR)
    return set_error(LBM_ERR_ARG, "tile_order = %d", p->tile_order);
  if (p->step_kernel < LBM_KERNEL_AUTO || p->step_kernel > LBM_KERNEL_SHUFFLE)
    return set_error(LBM_ERR_ARG, "step_kernel = %d", p->step_kernel);
  if (p->store_policy < LBM_STORE_AUTO || p->store_policy > LBM_STORE_NONTEMPORAL)
    return set_error(LBM_ERR_ARG, "store_policy = %d", p->store_policy);
  if (p->persistent != 0 && p->persistent != 1) return set_error(LBM_ERR_ARG, "persistent = %d", p->persistent);
  if (p->graph_steps < 0 || p->graph_steps > 100000)
    return set_error(LBM_ERR_ARG, "graph_steps = %d", p->graph_steps);
  if (p->model != LBM_MODEL_QUASI_COMPRESSIBLE && p->model != LBM_MODEL_INCOMPRESSIBLE)
    return set_error(LBM_ERR_ARG, "model = %d", p->model);
  if (p->pattern != LBM_PATTERN_TWO_COPY && p->pattern != LBM_PATTERN_SINGLE_COPY)
    return set_error(LBM_ERR_ARG, "pattern = %d", p->pattern);
  if (p->collision != LBM_COLLISION_BGK && p->collision != LBM_COLLISION_MRT)
    return set_error(LBM_ERR_ARG, "collision = %d", p->collision);
  if (p->reserved != 0) return set_error(LBM_ERR_ARG, "reserved field must be 0");
  for (int k = 0; k < 5; ++k)
    if (!(p->mrt_rates[k] == 0.0 || (p->mrt_rates[k] > 0.0 && p->mrt_rates[k] < 2.0)))
      return set_error(LBM_ERR_ARG, "mrt_rates[%d] = %g outside (0, 2)", k, p->mrt_rates[k]);
  int wpb = p->tiles_per_block == 0 ? 4 : p->tiles_per_block;
  if (p->lattice == 9) wpb = 4;  // a 16x16 tile is four wavefronts: one tile per workgroup
  v->q = p->lattice;
  v->ax = t->tile[0];
  v->ay = t->tile[1];
  v->az = t->tile[2];
  v->storage = p->storage;
  v->wpb = wpb;
  v->model = p->model;
  v->collision = p->collision;
  if (!lbm::variant_supported(*v))
    return set_error(LBM_ERR_UNSUPPORTED, "lattice D%dQ%d with tile %dx%dx%d and %d waves per block not built",
                     p->lattice == 9 ? 2 : 3, p->lattice, v->ax, v->ay, v->az, p->tiles_per_block);
  if (p->collision == LBM_COLLISION_MRT && (wpb != 4 || p->store_policy == LBM_STORE_REGULAR))
    return set_error(LBM_ERR_UNSUPPORTED, "the MRT collision is built for 4 waves per workgroup and non-temporal "
                                          "stores only");
  return LBM_OK;
}

int make_plan(const lbm_tiles *t, const lbm_params *p, const lbm::Variant &v, Plan &P) {
  const int q = v.q, sd = lbm::storage_bytes(v.storage), W = t->words;
  const int64_t A = 128 / sd;  // entries per 128-byte line
  const int64_t nft = t->n_ftiles;
  const double omega = std::isinf(p->tau) ? 0.0 : 1.0 / p->tau;
  try {
    // internal order: per sample, Morton order of tile coordinates (or row-major)
    std::vector<int64_t> perm((size_t)nft), inv((size_t)nft);
    for (int64_t k = 0; k < nft; ++k) perm[(size_t)k] = k;
    if (p->tile_order == LBM_ORDER_MORTON) {
      std::vector<uint64_t> key((size_t)nft);
      for (int64_t k = 0; k < nft; ++k)
        key[(size_t)k] = morton3((uint32_t)t->coord[(size_t)(3 * k)], (uint32_t)t->coord[(size_t)(3 * k + 1)],
                                 (uint32_t)t->coord[(size_t)(3 * k + 2)]);
      for (const lbm::Sample &S : t->samples)
        std::stable_sort(perm.begin() + S.tile0, perm.begin() + S.tile0 + S.n_ftiles,
                         [&](int64_t x, int64_t y) { return key[(size_t)x] < key[(size_t)y]; });
    }
    for (int64_t k = 0; k < nft; ++k) inv[(size_t)perm[(size_t)k]] = k;

    P.rec_h.resize((size_t)nft);
    P.fluid_h.resize((size_t)(nft * W));
    P.pre_h.resize((size_t)(nft * W));
    P.nbr_h.resize((size_t)(nft * 27));
    P.coord_h.resize((size_t)(nft * 3));
    P.nbase_h.resize((size_t)nft);
    int64_t off = 0, nb = 0;
    for (int64_t k = 0; k < nft; ++k) {
      const int64_t c = perm[(size_t)k];  // canonical index of internal tile k
      int n = 0;
      for (int w = 0; w < W; ++w) {
        const uint64_t m = t->fluid[(size_t)(c * W + w)];
        P.fluid_h[(size_t)(k * W + w)] = m;
        P.pre_h[(size_t)(k * W + w)] = n;
        n += __builtin_popcountll(m);
      }
      for (int j = 0; j < 27; ++j) {
        const int32_t o = t->nbr[(size_t)(c * 27 + j)];
        P.nbr_h[(size_t)(k * 27 + j)] = o < 0 ? -1 : (int32_t)inv[(size_t)o];
      }
      for (int a = 0; a < 3; ++a) P.coord_h[(size_t)(k * 3 + a)] = t->coord[(size_t)(c * 3 + a)];
      P.rec_h[(size_t)k] = lbm::TileRec{off, n, t->sample_of[(size_t)c]};
      P.nbase_h[(size_t)k] = nb;
      off += ((int64_t)q * n + A - 1) / A * A;
      nb += n;
    }
    P.entries = off;
    // Records of the scalar-mask D3Q19 kernel, one per wavefront: a 4x4x4
    // tile, or one 4x4x4 half (z < 4, z >= 4) of a 4x4x8 tile.  A half's
    // record holds its own fluid mask and its first entry (the tile's offset,
    // plus the lower half's fluid nodes for the upper half), and the tile's
    // node count as the stride between direction blocks, so the kernel's
    // arithmetic is the same for both shapes.
    const bool halves = W == 2 && v.ax == 4 && v.ay == 4 && v.az == 8;
    const int64_t nw = nft * W;  // wavefronts
    if (q == 19 && (W == 1 || halves)) {
      P.nrec_h.resize((size_t)nw + 1);
      // neighbour rows hold byte offsets into the record array (the sentinel
      // record for a missing neighbour), so the kernel adds them to the base
      // pointer without a 64-bit multiply
      if ((uint64_t)(nw + 1) * sizeof(lbm::NbRec) > UINT32_MAX)
        return set_error(LBM_ERR_UNSUPPORTED, "too many tiles (%lld) for 32-bit record offsets", (long long)nft);
      const uint32_t sentinel = (uint32_t)((uint64_t)nw * sizeof(lbm::NbRec));
      P.nrow_h.assign((size_t)(nw * 20), sentinel);
      for (int64_t k = 0; k < nft; ++k) {
        const lbm::TileRec &r = P.rec_h[(size_t)k];
        int lower = 0;  // fluid nodes of the halves below this one
        for (int h = 0; h < W; ++h) {
          const int64_t wv = k * W + h;
          const uint64_t m = P.fluid_h[(size_t)(k * W + h)];
          P.nrec_h[(size_t)wv] = lbm::NbRec{(uint32_t)(r.off + lower), (uint32_t)r.n, m, r.sample, 0};
          lower += __builtin_popcountll(m);
          for (int j = 0; j < 18; ++j) {
            // slot (dx, dy, dz) of the 3x3x3 neighbourhood in units of 4x4x4 wavefront tiles
            const int sl = kGatherSlots[j], dx = sl % 3 - 1, dy = (sl / 3) % 3 - 1, dz = sl / 9 - 1;
            const int hz = h + dz;                            // neighbour half along z
            const int tdz = hz < 0 ? -1 : (hz >= W ? 1 : 0);  // tile step along z
            const int nh = hz - tdz * W;
            const int32_t o = P.nbr_h[(size_t)(k * 27 + (dx + 1) + 3 * (dy + 1) + 9 * (tdz + 1))];
            P.nrow_h[(size_t)(wv * 20 + j)] =
                o < 0 ? sentinel : (uint32_t)((uint64_t)((int64_t)o * W + nh) * sizeof(lbm::NbRec));
          }
        }
      }
      P.nrec_h[(size_t)nw] = lbm::NbRec{0u, 0u, 0ull, 0, 0};
      // region bases: off + b*n of the region's source tile (b the slot the
      // gather reads: i, or opp(i) for the single copy), plus the fluid nodes
      // that the shift to the destination lanes moves out below lane 0 (the
      // kernel adds v_mbcnt of the shifted mask); 0 for a missing source.
      // Only the FP16 form reads them.  For FP32 the table (read with the
      // loads kept where their addresses are ready, or without) measured
      // 17-30% slower than computing the bases, and as 16-bit entries
      // relative to the source tile 37% slower; FP64 is bound by bytes.
      if (p->storage == LBM_F16_OFFSET) P.rbase_h.assign((size_t)(nw * lbm::kRegionBases), 0u);
      for (int64_t k = 0; k < nw && !P.rbase_h.empty(); ++k) {
        uint32_t *rb = &P.rbase_h[(size_t)(k * lbm::kRegionBases)];
        for (int i = 1; i < 19; ++i) {
          const int cx = lbm::D3Q19::C[i][0], cy = lbm::D3Q19::C[i][1], cz = lbm::D3Q19::C[i][2];
          const int d0 = cx + 4 * cy + 16 * cz;
          for (int w = 0; w < 8; ++w) {
            if (!lbm::region_valid(i, w)) continue;
            const int wx = w & 1, wy = (w >> 1) & 1, wz = (w >> 2) & 1;
            const int dr = d0 - (wx ? 4 * cx : 0) - (wy ? 16 * cy : 0) - (wz ? 64 * cz : 0);
            const lbm::NbRec *r = &P.nrec_h[(size_t)k];
            if (w != 0) {
              const int slot = 13 + (wx ? -cx : 0) + 3 * (wy ? -cy : 0) + 9 * (wz ? -cz : 0);
              int j = 0;
              while (kGatherSlots[j] != slot) ++j;
              r = &P.nrec_h[P.nrow_h[(size_t)(k * 20 + j)] / sizeof(lbm::NbRec)];
            }
            const uint32_t dropped =
                dr >= 0 ? 0u : (uint32_t)__builtin_popcountll(r->mask & ((1ull << (-dr)) - 1ull));
            const int b = p->pattern == LBM_PATTERN_SINGLE_COPY ? lbm::D3Q19::Opp[i] : i;
            rb[lbm::region_index(i, w)] = r->off + (uint32_t)b * r->n + dropped;
          }
        }
      }
    }
    P.samples_h.resize(t->samples.size());
    P.coef_h.resize(t->samples.size());
    for (size_t s = 0; s < t->samples.size(); ++s) {
      const lbm::Sample &S = t->samples[s];
      lbm::SampleRec &R = P.samples_h[s];
      std::memset(&R, 0, sizeof R);
      for (int a = 0; a < 3; ++a) {
        R.g[a] = p->g[a];
        R.shape[a] = S.shape[a];
      }
      R.dense0 = S.dense0;
      R.n_nodes = S.n_nodes;
      R.tile0 = S.tile0;
      R.n_ftiles = S.n_ftiles;
      R.nbase0 = S.n_ftiles ? P.nbase_h[(size_t)S.tile0] : 0;
      R.n_fluid = S.n_fluid;
      fill_coef(P.coef_h[s], p->g, omega);
    }
  } catch (const std::bad_alloc &) {
    return set_error(LBM_ERR_NOMEM, "out of host memory planning the workspace");
  }
  const int64_t waves = nft * W;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, kAlign);
    return at;
  };
  P.buf[0] = take((size_t)P.entries * sd);
  P.buf[1] = p->pattern == LBM_PATTERN_SINGLE_COPY ? P.buf[0] : take((size_t)P.entries * sd);
  P.rec = take((size_t)nft * sizeof(lbm::TileRec));
  P.fluid = take((size_t)(nft * W) * sizeof(uint64_t));
  P.pre = take((size_t)(nft * W) * sizeof(int32_t));
  P.nbr = take((size_t)(nft * 27) * sizeof(int32_t));
  P.coord = take((size_t)(nft * 3) * sizeof(int32_t));
  P.nbase = take((size_t)nft * sizeof(int64_t));
  P.samples = take(t->samples.size() * sizeof(lbm::SampleRec));
  P.coef = take(t->samples.size() * sizeof(lbm::CollideCoef));
  P.nrec = take(P.nrec_h.size() * sizeof(lbm::NbRec));
  P.nrow = take(P.nrow_h.size() * sizeof(uint32_t));
  P.rbase = take(P.rbase_h.size() * sizeof(uint32_t));
  P.list = take((size_t)(nft > 0 ? nft * W : 1) * sizeof(int32_t));
  P.lid = take((size_t)(nft > 0 ? nft : 1) * sizeof(int32_t));
  P.count = take(sizeof(int32_t));
  P.part = take((size_t)(waves > 0 ? waves : 1) * 4 * sizeof(double));
  P.chunk = take(t->samples.size() * (size_t)lbm::reduce_chunks() * 4 * sizeof(double));
  P.out = take(t->samples.size() * 4 * sizeof(double));
  P.uref = take((size_t)(3 * (t->n_fluid > 0 ? t->n_fluid : 1)) * sizeof(double));
  P.total = o;
  return LBM_OK;
}

}  // namespace

struct lbm_solver {
  lbm::Variant var{};
  lbm_params p{};
  hipStream_t stream = nullptr;
  lbm::TileArgs args{};
  void *buf[2] = {nullptr, nullptr};  // the same buffer twice for the single copy
  bool single_copy = false;
  int cur = 0;  // two copies: the copy holding the state; single copy: its layout (0 or 1)
  int64_t steps = 0;
  bool initialized = false;
  int n_samples = 0;
  int words = 0;
  double omega = 0.0;
  int64_t dense_nodes = 0;
  std::vector<lbm::SampleRec> samples_h;
  lbm::SampleRec *samples_d = nullptr;
  std::vector<uint32_t> periodic;  // per sample
  std::vector<lbm::CollideCoef> coef_h;
  lbm::CollideCoef *coef_d = nullptr;
  const lbm::NbRec *nrec_d = nullptr;
  const uint32_t *nrow_d = nullptr;
  const uint32_t *rbase_d = nullptr;
  // active tile list (batches) and the launch mode of the scalar-mask step
  int32_t *list_d = nullptr, *count_d = nullptr;
  // moving wall: tiles holding the lattice's first or last row along its axis
  int32_t *lid_tiles_d = nullptr;
  int64_t n_lid_tiles = 0;
  std::vector<int32_t> list_h;
  int32_t count_h = 0;
  std::vector<uint8_t> active_h;
  bool all_active = true;
  int64_t persistent_blocks = 0;
  // per sample: [first, last) PDF entry of its tiles' regions
  std::vector<int64_t> entry0, entry1;
  int storage_bytes = 8;
  // captured graphs of graph_steps steps, one per starting copy
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  bool scalar_mask = false;  // which step kernel runs
  bool shuffle = false;      // the scalar-mask kernel in its shuffle form
  double *part = nullptr, *chunk = nullptr, *out = nullptr, *uref = nullptr;
  std::vector<double> out_h;
};

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return set_error(LBM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

extern "C" int lbm_lattice(int32_t q, int32_t *c, double *w, int32_t *opp) {
  if (!c || !w || !opp) return set_error(LBM_ERR_ARG, "lbm_lattice: NULL argument");
  auto fill = [&](const auto &L) {
    using LT = std::decay_t<decltype(L)>;
    for (int i = 0; i < LT::Q; ++i) {
      for (int a = 0; a < 3; ++a) c[3 * i + a] = LT::C[i][a];
      w[i] = LT::Wt[i];
      opp[i] = LT::Opp[i];
    }
  };
  if (q == 9)
    fill(lbm::D2Q9{});
  else if (q == 19)
    fill(lbm::D3Q19{});
  else
    return set_error(LBM_ERR_UNSUPPORTED, "lbm_lattice: q = %d", q);
  return LBM_OK;
}

extern "C" int lbm_workspace_bytes(const lbm_tiles *t, const lbm_params *p, size_t *bytes) {
  if (!bytes) return set_error(LBM_ERR_ARG, "lbm_workspace_bytes: NULL bytes");
  lbm::Variant v;
  int rc = check_params(t, p, &v);
  if (rc) return rc;
  Plan P;
  rc = make_plan(t, p, v, P);
  if (rc) return rc;
  *bytes = P.total;
  return LBM_OK;
}

extern "C" int lbm_create(const lbm_tiles *t, const lbm_params *p, void *ws, size_t bytes, void *stream,
                          lbm_solver **out) {
  if (!out) return set_error(LBM_ERR_ARG, "lbm_create: NULL out");
  *out = nullptr;
  lbm::Variant v;
  int rc = check_params(t, p, &v);
  if (rc) return rc;
  if (!ws) return set_error(LBM_ERR_ARG, "lbm_create: NULL workspace");
  if ((uintptr_t)ws % kAlign) return set_error(LBM_ERR_ARG, "lbm_create: workspace not %zu-byte aligned", kAlign);
  Plan P;
  rc = make_plan(t, p, v, P);
  if (rc) return rc;
  if (bytes < P.total)
    return set_error(LBM_ERR_NOMEM, "lbm_create: workspace of %zu bytes, %zu needed", bytes, P.total);

  lbm_solver *s = new (std::nothrow) lbm_solver();
  if (!s) return set_error(LBM_ERR_NOMEM, "lbm_create: out of host memory");
  char *base = static_cast<char *>(ws);
  s->var = v;
  s->p = *p;
  s->stream = static_cast<hipStream_t>(stream);
  s->buf[0] = base + P.buf[0];
  s->buf[1] = base + P.buf[1];
  s->single_copy = p->pattern == LBM_PATTERN_SINGLE_COPY;
  s->n_samples = (int)t->samples.size();
  s->words = t->words;
  s->omega = std::isinf(p->tau) ? 0.0 : 1.0 / p->tau;
  s->dense_nodes = t->n_nodes;
  s->samples_h = P.samples_h;
  s->samples_d = reinterpret_cast<lbm::SampleRec *>(base + P.samples);
  s->coef_h = P.coef_h;
  s->coef_d = reinterpret_cast<lbm::CollideCoef *>(base + P.coef);
  s->nrec_d = reinterpret_cast<const lbm::NbRec *>(base + P.nrec);
  s->nrow_d = reinterpret_cast<const uint32_t *>(base + P.nrow);
  s->rbase_d = reinterpret_cast<const uint32_t *>(base + P.rbase);
  s->list_d = reinterpret_cast<int32_t *>(base + P.list);
  s->lid_tiles_d = reinterpret_cast<int32_t *>(base + P.lid);
  s->count_d = reinterpret_cast<int32_t *>(base + P.count);
  s->storage_bytes = lbm::storage_bytes(v.storage);
  try {
    // the active list counts wavefronts: tiles, or the 4x4x4 halves of 4x4x8 tiles
    s->list_h.resize((size_t)(t->n_ftiles * t->words));
    for (int64_t k = 0; k < t->n_ftiles * t->words; ++k) s->list_h[(size_t)k] = (int32_t)k;
    s->count_h = (int32_t)(t->n_ftiles * t->words);
    s->active_h.assign(t->samples.size(), 1);
    for (const lbm::Sample &S : t->samples) s->periodic.push_back(S.periodic);
    for (const lbm::Sample &S : t->samples) {
      if (S.n_ftiles == 0) {
        s->entry0.push_back(0);
        s->entry1.push_back(0);
        continue;
      }
      const lbm::TileRec &a0 = P.rec_h[(size_t)S.tile0], &a1 = P.rec_h[(size_t)(S.tile0 + S.n_ftiles - 1)];
      const int64_t A = 128 / s->storage_bytes;
      s->entry0.push_back(a0.off);
      s->entry1.push_back(a1.off + ((int64_t)v.q * a1.n + A - 1) / A * A);
    }
  } catch (const std::bad_alloc &) {
    delete s;
    return set_error(LBM_ERR_NOMEM, "lbm_create: out of host memory");
  }
  const bool fits32 = P.entries < (int64_t(1) << 32);
  if ((p->step_kernel == LBM_KERNEL_SCALAR_MASK || p->step_kernel == LBM_KERNEL_SHUFFLE) &&
      !(lbm::step19_supported(v) && fits32)) {
    delete s;
    return set_error(LBM_ERR_UNSUPPORTED, "lbm_create: the scalar-mask and shuffle kernels need D3Q19, 4x4x4 or "
                                          "4x4x8 tiles and fewer than 2^32 PDF entries per copy");
  }
  if (p->step_kernel == LBM_KERNEL_SHUFFLE && p->pattern != LBM_PATTERN_TWO_COPY) {
    delete s;
    return set_error(LBM_ERR_UNSUPPORTED, "lbm_create: the shuffle kernel is a two-copy step");
  }
  // automatic choice: the scalar-mask kernel for 4x4x4 tiles; for 4x4x8 tiles
  // only when asked for
  s->scalar_mask = (p->step_kernel == LBM_KERNEL_AUTO ? v.az == 4 : p->step_kernel != LBM_KERNEL_GENERIC) &&
                   lbm::step19_supported(v) && fits32;
  s->shuffle = p->step_kernel == LBM_KERNEL_SHUFFLE;
  if (p->persistent && !s->scalar_mask) {
    delete s;
    return set_error(LBM_ERR_UNSUPPORTED, "lbm_create: the persistent step needs the scalar-mask D3Q19 kernel");
  }
  s->part = reinterpret_cast<double *>(base + P.part);
  s->chunk = reinterpret_cast<double *>(base + P.chunk);
  s->out = reinterpret_cast<double *>(base + P.out);
  s->uref = reinterpret_cast<double *>(base + P.uref);
  s->out_h.assign((size_t)s->n_samples * 4, 0.0);

  lbm::TileArgs &a = s->args;
  a.rec = reinterpret_cast<const lbm::TileRec *>(base + P.rec);
  a.fluid = reinterpret_cast<const uint64_t *>(base + P.fluid);
  a.pre = reinterpret_cast<const int32_t *>(base + P.pre);
  a.nbr = reinterpret_cast<const int32_t *>(base + P.nbr);
  a.coord = reinterpret_cast<const int32_t *>(base + P.coord);
  a.nbase = reinterpret_cast<const int64_t *>(base + P.nbase);
  a.samples = s->samples_d;
  a.n_waves = t->n_ftiles * t->words;
  a.n_fluid = t->n_fluid;
  a.rho0 = p->rho0;
  a.model = p->model;
  a.aa_phase = s->single_copy ? 0 : -1;
  a.mrt = mrt_rates(p, s->omega);
  a.lid.axis = -1;
  a.lid.side = 0;
  a.f16_scale = std::ldexp(1.0f, p->f16_scale_log2);
  a.f16_inv = std::ldexp(1.0f, -p->f16_scale_log2);

  auto up = [&](size_t off, const void *src, size_t n) -> hipError_t {
    if (n == 0) return hipSuccess;
    return hipMemcpyAsync(base + off, src, n, hipMemcpyHostToDevice, s->stream);
  };
  hipError_t e = hipSuccess;
  const int64_t nft = t->n_ftiles, W = t->words;
  if (e == hipSuccess) e = up(P.rec, P.rec_h.data(), (size_t)nft * sizeof(lbm::TileRec));
  if (e == hipSuccess) e = up(P.fluid, P.fluid_h.data(), (size_t)(nft * W) * sizeof(uint64_t));
  if (e == hipSuccess) e = up(P.pre, P.pre_h.data(), (size_t)(nft * W) * sizeof(int32_t));
  if (e == hipSuccess) e = up(P.nbr, P.nbr_h.data(), (size_t)(nft * 27) * sizeof(int32_t));
  if (e == hipSuccess) e = up(P.coord, P.coord_h.data(), (size_t)(nft * 3) * sizeof(int32_t));
  if (e == hipSuccess) e = up(P.coef, P.coef_h.data(), P.coef_h.size() * sizeof(lbm::CollideCoef));
  if (e == hipSuccess) e = up(P.nrec, P.nrec_h.data(), P.nrec_h.size() * sizeof(lbm::NbRec));
  if (e == hipSuccess) e = up(P.nrow, P.nrow_h.data(), P.nrow_h.size() * sizeof(uint32_t));
  if (e == hipSuccess) e = up(P.rbase, P.rbase_h.data(), P.rbase_h.size() * sizeof(uint32_t));
  if (e == hipSuccess) e = up(P.list, s->list_h.data(), s->list_h.size() * sizeof(int32_t));
  if (e == hipSuccess) e = up(P.count, &s->count_h, sizeof(int32_t));
  if (e == hipSuccess && s->scalar_mask && p->persistent)
    e = lbm::step19_persistent_blocks(v, s->single_copy, s->shuffle, &s->persistent_blocks);
  if (e == hipSuccess) e = up(P.nbase, P.nbase_h.data(), (size_t)nft * sizeof(int64_t));
  if (e == hipSuccess) e = up(P.samples, P.samples_h.data(), P.samples_h.size() * sizeof(lbm::SampleRec));
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);  // host tables may be freed after return
  if (e != hipSuccess) {
    delete s;
    return set_error(LBM_ERR_HIP, "lbm_create: upload failed: %s", hipGetErrorString(e));
  }
  *out = s;
  return LBM_OK;
}

static void drop_graphs(lbm_solver *s) {
  for (hipGraphExec_t &g : s->graph)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

extern "C" void lbm_destroy(lbm_solver *s) {
  if (!s) return;
  drop_graphs(s);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  delete s;
}

extern "C" int lbm_set_stream(lbm_solver *s, void *stream) {
  if (!s) return set_error(LBM_ERR_ARG, "lbm_set_stream: NULL solver");
  s->stream = static_cast<hipStream_t>(stream);
  return LBM_OK;
}

extern "C" int lbm_set_active(lbm_solver *s, const uint8_t *active) {
  if (!s || !active) return set_error(LBM_ERR_ARG, "lbm_set_active: NULL argument");
  if (!s->scalar_mask)
    return set_error(LBM_ERR_UNSUPPORTED, "lbm_set_active: needs the scalar-mask D3Q19 kernel (4x4x4 tiles)");
  bool changed = false;
  for (int k = 0; k < s->n_samples; ++k) changed |= (s->active_h[(size_t)k] != 0) != (active[k] != 0);
  // single copy: frozen samples are kept in layout 0, which active samples
  // share only after an even number of steps
  if (s->single_copy && changed && s->cur != 0)
    return set_error(LBM_ERR_STATE, "lbm_set_active: with one PDF copy the active set may change only after an "
                                    "even number of steps");
  // samples that stop here: make both PDF copies hold their current state
  for (int k = 0; k < s->n_samples && !s->single_copy; ++k) {
    if (s->active_h[(size_t)k] && !active[k] && s->initialized && s->entry1[(size_t)k] > s->entry0[(size_t)k]) {
      const size_t off = (size_t)s->entry0[(size_t)k] * s->storage_bytes;
      const size_t len = (size_t)(s->entry1[(size_t)k] - s->entry0[(size_t)k]) * s->storage_bytes;
      HIP_TRY(hipMemcpyAsync(static_cast<char *>(s->buf[s->cur ^ 1]) + off, static_cast<char *>(s->buf[s->cur]) + off,
                             len, hipMemcpyDeviceToDevice, s->stream));
    }
  }
  int32_t n = 0;
  bool all = true;
  for (int k = 0; k < s->n_samples; ++k) {
    s->active_h[(size_t)k] = active[k] ? 1 : 0;
    s->samples_h[(size_t)k].frozen = active[k] ? 0 : 1;
    all &= active[k] != 0;
    if (!active[k]) continue;
    const lbm::SampleRec &S = s->samples_h[(size_t)k];
    for (int64_t w = S.tile0 * s->words; w < (S.tile0 + S.n_ftiles) * s->words; ++w)
      s->list_h[(size_t)n++] = (int32_t)w;
  }
  s->count_h = n;
  HIP_TRY(hipMemcpyAsync(s->list_d, s->list_h.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(s->count_d, &s->count_h, sizeof(int32_t), hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(s->samples_d, s->samples_h.data(), s->samples_h.size() * sizeof(lbm::SampleRec),
                         hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  // the non-persistent step switches between direct and list-driven launches
  // here, so its captured graphs no longer match
  if (!s->p.persistent && s->all_active != all) drop_graphs(s);
  s->all_active = all;
  return LBM_OK;
}

extern "C" int lbm_set_lid(lbm_solver *s, int32_t axis, int32_t side, const double *u) {
  if (!s) return set_error(LBM_ERR_ARG, "lbm_set_lid: NULL solver");
  lbm::LidArgs &L = s->args.lid;
  if (axis == -1) {
    L.axis = -1;
    s->n_lid_tiles = 0;
    drop_graphs(s);
    return LBM_OK;
  }
  if (!u) return set_error(LBM_ERR_ARG, "lbm_set_lid: NULL u");
  if (axis < 0 || axis > 2 || (s->var.q == 9 && axis == 2))
    return set_error(LBM_ERR_ARG, "lbm_set_lid: axis = %d", axis);
  if (side != 0 && side != 1) return set_error(LBM_ERR_ARG, "lbm_set_lid: side = %d", side);
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(u[a])) return set_error(LBM_ERR_ARG, "lbm_set_lid: u[%d] not finite", a);
  for (size_t k = 0; k < s->periodic.size(); ++k)
    if ((s->periodic[k] >> axis) & 1u)
      return set_error(LBM_ERR_ARG, "lbm_set_lid: axis %d is periodic in sample %zu", axis, k);
  const double rho_w = s->p.model == LBM_MODEL_INCOMPRESSIBLE ? 1.0 : s->p.rho0;
  for (int i = 0; i < 19; ++i) {
    double cu = 0.0, w = 0.0;
    if (s->var.q == 9 && i < 9) {
      cu = lbm::D2Q9::C[i][0] * u[0] + lbm::D2Q9::C[i][1] * u[1];
      w = lbm::D2Q9::Wt[i];
    } else if (s->var.q == 19) {
      cu = lbm::D3Q19::C[i][0] * u[0] + lbm::D3Q19::C[i][1] * u[1] + lbm::D3Q19::C[i][2] * u[2];
      w = lbm::D3Q19::Wt[i];
    }
    L.corr[i] = 6.0 * w * rho_w * cu;
    L.corrf[i] = (float)L.corr[i];
  }
  // the tiles that hold the lid row of their sample (tile tables back from the device)
  const int64_t nft = s->args.n_waves / s->words;
  std::vector<int32_t> coord, lid;
  std::vector<lbm::TileRec> rec;
  try {
    coord.resize((size_t)(3 * nft));
    rec.resize((size_t)nft);
  } catch (const std::bad_alloc &) {
    return set_error(LBM_ERR_NOMEM, "lbm_set_lid: out of host memory");
  }
  if (nft > 0) {
    HIP_TRY(hipMemcpyAsync(coord.data(), s->args.coord, coord.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                           s->stream));
    HIP_TRY(hipMemcpyAsync(rec.data(), s->args.rec, rec.size() * sizeof(lbm::TileRec), hipMemcpyDeviceToHost,
                           s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  }
  const int edge = axis == 0 ? s->var.ax : axis == 1 ? s->var.ay : s->var.az;
  for (int64_t k = 0; k < nft; ++k) {
    const int n = s->samples_h[(size_t)rec[(size_t)k].sample].shape[axis];
    const int row = side ? n - 1 : 0, t0 = coord[(size_t)(3 * k + axis)] * edge;
    if (row >= t0 && row < t0 + edge) lid.push_back((int32_t)k);
  }
  if (!lid.empty()) {
    HIP_TRY(hipMemcpyAsync(s->lid_tiles_d, lid.data(), lid.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  }
  s->n_lid_tiles = (int64_t)lid.size();
  L.axis = axis;
  L.side = side;
  drop_graphs(s);  // captured launches hold the old arguments
  return LBM_OK;
}

extern "C" int lbm_set_sample_force(lbm_solver *s, const double *g) {
  if (!s || !g) return set_error(LBM_ERR_ARG, "lbm_set_sample_force: NULL argument");
  for (int k = 0; k < 3 * s->n_samples; ++k)
    if (!std::isfinite(g[k])) return set_error(LBM_ERR_ARG, "lbm_set_sample_force: g[%d] not finite", k);
  for (int k = 0; k < s->n_samples; ++k) {
    for (int a = 0; a < 3; ++a) s->samples_h[(size_t)k].g[a] = g[3 * k + a];
    fill_coef(s->coef_h[(size_t)k], &g[3 * k], s->omega);
  }
  HIP_TRY(hipMemcpyAsync(s->samples_d, s->samples_h.data(), s->samples_h.size() * sizeof(lbm::SampleRec),
                         hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(s->coef_d, s->coef_h.data(), s->coef_h.size() * sizeof(lbm::CollideCoef),
                         hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return LBM_OK;
}

// Layout of the state for the auxiliary kernels.
static lbm::TileArgs &aux_args(lbm_solver *s) {
  s->args.aa_phase = s->single_copy ? s->cur : -1;
  return s->args;
}

extern "C" int lbm_init(lbm_solver *s, const double *rho, const double *u) {
  if (!s) return set_error(LBM_ERR_ARG, "lbm_init: NULL solver");
  s->cur = 0;
  HIP_TRY(lbm::launch_init(s->var, s->buf[0], aux_args(s), rho, u, s->stream));
  s->steps = 0;
  s->initialized = true;
  // record the reference velocity of the residual
  HIP_TRY(lbm::launch_residual_partial(s->var, s->buf[0], aux_args(s), s->uref, s->part, 0, s->stream));
  return LBM_OK;
}

// Enqueue one step from copy (two copies) or layout (single copy) `from` on `st`.
static hipError_t enqueue_step(lbm_solver *s, int from, hipStream_t st) {
  const int phase = !s->single_copy ? lbm::kPhaseTwoCopy : (from == 0 ? lbm::kPhaseAAGather : lbm::kPhaseAALocal);
  if (s->args.lid.axis >= 0 && s->n_lid_tiles > 0) {
    const hipError_t e =
        lbm::launch_lid_fixup(s->var, s->buf[from], s->args, s->lid_tiles_d, s->n_lid_tiles, s->single_copy, st);
    if (e != hipSuccess) return e;
  }
  if (s->scalar_mask) {
    const int mode = s->p.persistent ? 2 : (s->all_active ? 0 : 1);
    return lbm::launch_step19(s->var, phase, s->shuffle, s->buf[from], s->buf[from ^ 1], s->args, s->nrec_d, s->nrow_d,
                              s->rbase_d, s->coef_d, s->p.store_policy != LBM_STORE_REGULAR, s->list_d, s->count_d,
                              mode, s->persistent_blocks, st);
  }
  return lbm::launch_step(s->var, phase, s->buf[from], s->buf[from ^ 1], s->args, s->omega, st);
}

// Capture graph_steps steps starting from copy `from` (on a private stream:
// the caller's stream may be the null stream, which cannot be captured).
static int capture(lbm_solver *s, int from) {
  if (!s->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  int c = from;
  for (int k = 0; k < s->p.graph_steps && e == hipSuccess; ++k) {
    e = enqueue_step(s, c, s->cap_stream);
    c ^= 1;
  }
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(s->cap_stream, &g);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&s->graph[from], g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) return set_error(LBM_ERR_HIP, "lbm_step: graph capture failed: %s", hipGetErrorString(e));
  return LBM_OK;
}

extern "C" int lbm_step(lbm_solver *s, int32_t n) {
  if (!s) return set_error(LBM_ERR_ARG, "lbm_step: NULL solver");
  if (n < 0) return set_error(LBM_ERR_ARG, "lbm_step: n = %d", n);
  if (!s->initialized) return set_error(LBM_ERR_STATE, "lbm_step: call lbm_init or lbm_pdfs_import first");
  const int K = s->p.graph_steps;
  if (K > 0 && s->args.n_waves > 0) {
    while (n >= K) {
      if (!s->graph[s->cur]) {
        const int rc = capture(s, s->cur);
        if (rc) return rc;
      }
      HIP_TRY(hipGraphLaunch(s->graph[s->cur], s->stream));
      s->cur ^= (K & 1);
      s->steps += K;
      n -= K;
    }
  }
  for (int32_t k = 0; k < n; ++k) {
    HIP_TRY(enqueue_step(s, s->cur, s->stream));
    s->cur ^= 1;
    ++s->steps;
  }
  return LBM_OK;
}

extern "C" int64_t lbm_step_count(const lbm_solver *s) { return s ? s->steps : -1; }

extern "C" int lbm_moments(lbm_solver *s, double *rho, double *u) {
  if (!s) return set_error(LBM_ERR_ARG, "lbm_moments: NULL solver");
  if (!s->initialized) return set_error(LBM_ERR_STATE, "lbm_moments: solver not initialised");
  if (rho) HIP_TRY(lbm::launch_fill(rho, s->dense_nodes, 0.0, s->stream));
  if (u) HIP_TRY(lbm::launch_fill(u, 3 * s->dense_nodes, 0.0, s->stream));
  HIP_TRY(lbm::launch_moments(s->var, s->buf[s->cur], aux_args(s), rho, u, s->stream));
  return LBM_OK;
}

extern "C" int lbm_reduce(lbm_solver *s, double *out_host) {
  if (!s || !out_host) return set_error(LBM_ERR_ARG, "lbm_reduce: NULL argument");
  if (!s->initialized) return set_error(LBM_ERR_STATE, "lbm_reduce: solver not initialised");
  HIP_TRY(lbm::launch_reduce_partial(s->var, s->buf[s->cur], aux_args(s), s->part, s->stream));
  HIP_TRY(lbm::launch_reduce_final(s->part, 4, s->samples_d, s->n_samples, s->words, s->chunk, s->out,
                                     s->stream));
  HIP_TRY(hipMemcpyAsync(s->out_h.data(), s->out, (size_t)s->n_samples * 4 * sizeof(double),
                         hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  std::memcpy(out_host, s->out_h.data(), (size_t)s->n_samples * 4 * sizeof(double));
  for (int k = 0; k < 4 * s->n_samples; ++k)
    if (!std::isfinite(out_host[k])) return set_error(LBM_ERR_NONFINITE, "lbm_reduce: total %d is not finite", k);
  return LBM_OK;
}

extern "C" int lbm_residual(lbm_solver *s, double *out_host) {
  if (!s || !out_host) return set_error(LBM_ERR_ARG, "lbm_residual: NULL argument");
  if (!s->initialized) return set_error(LBM_ERR_STATE, "lbm_residual: solver not initialised");
  HIP_TRY(lbm::launch_residual_partial(s->var, s->buf[s->cur], aux_args(s), s->uref, s->part, 1, s->stream));
  HIP_TRY(lbm::launch_reduce_final(s->part, 2, s->samples_d, s->n_samples, s->words, s->chunk, s->out,
                                     s->stream));
  HIP_TRY(hipMemcpyAsync(s->out_h.data(), s->out, (size_t)s->n_samples * 2 * sizeof(double),
                         hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  int bad = -1;
  for (int k = 0; k < s->n_samples; ++k) {
    const double d2 = s->out_h[(size_t)(2 * k)], n2 = s->out_h[(size_t)(2 * k + 1)];
    double r;
    if (n2 > 0.0)
      r = std::sqrt(d2 / n2);
    else
      r = d2 > 0.0 ? INFINITY : 0.0;
    if (!std::isfinite(d2) || !std::isfinite(n2)) {
      r = NAN;
      bad = k;
    }
    out_host[k] = r;
  }
  if (bad >= 0) return set_error(LBM_ERR_NONFINITE, "lbm_residual: sample %d is not finite", bad);
  return LBM_OK;
}

extern "C" int lbm_pdfs_export(lbm_solver *s, double *dev_dense) {
  if (!s || !dev_dense) return set_error(LBM_ERR_ARG, "lbm_pdfs_export: NULL argument");
  if (!s->initialized) return set_error(LBM_ERR_STATE, "lbm_pdfs_export: solver not initialised");
  HIP_TRY(lbm::launch_fill(dev_dense, (int64_t)s->var.q * s->dense_nodes, 0.0, s->stream));
  HIP_TRY(lbm::launch_export(s->var, s->buf[s->cur], aux_args(s), dev_dense, s->stream));
  return LBM_OK;
}

extern "C" int lbm_pdfs_import(lbm_solver *s, const double *dev_dense) {
  if (!s || !dev_dense) return set_error(LBM_ERR_ARG, "lbm_pdfs_import: NULL argument");
  if (s->single_copy) s->cur = 0;  // import writes layout 0
  HIP_TRY(lbm::launch_import(s->var, s->buf[s->cur], aux_args(s), dev_dense, s->stream));
  s->initialized = true;
  return LBM_OK;
}
