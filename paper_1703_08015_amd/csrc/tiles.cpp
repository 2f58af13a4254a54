// Host tiling of a solid mask (arXiv 1703.08015, Sec. 3): a uniform mesh of
// fixed-size tiles starting at node (0, 0); non-periodic axes are extended
// with solid nodes up to a multiple of the tile edge; tiles holding only
// solid nodes are dropped.  The tile map stores the index of each non-empty
// tile and -1 for empty ones (two-copy method, Sec. 3); each non-empty tile
// also gets its 27-entry neighbour row (the 3x3x3 tile neighbourhood the
// gather kernel of Fig. 5 consults), with periodic axes wrapped.
//
// One O(N) pass over the mask builds per-tile fluid bitmasks for all tiles;
// a second pass over the tile grid compacts the non-empty ones.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.h"

namespace lbm {

namespace {
thread_local std::string g_error;
}

int set_error(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

const char *last_error() { return g_error.c_str(); }

static bool tile_supported(const int32_t t[3]) {
  return (t[0] == 4 && t[1] == 4 && t[2] == 4) || (t[0] == 4 && t[1] == 4 && t[2] == 8) ||
         (t[0] == 16 && t[1] == 16 && t[2] == 1);
}

}  // namespace lbm

using lbm::set_error;

extern "C" int lbm_tiles_build(const uint8_t *solid, const int32_t shape[3], const int32_t tile[3],
                               uint32_t periodic, lbm_tiles **out) {
  if (!solid || !shape || !tile || !out) return set_error(LBM_ERR_ARG, "lbm_tiles_build: NULL argument");
  *out = nullptr;
  if (!lbm::tile_supported(tile))
    return set_error(LBM_ERR_UNSUPPORTED, "lbm_tiles_build: tile %dx%dx%d not supported (4x4x4, 4x4x8, 16x16x1)",
                     tile[0], tile[1], tile[2]);
  if (periodic > 7u) return set_error(LBM_ERR_ARG, "lbm_tiles_build: periodic bits %u", periodic);
  int64_t n[3], np[3], T[3];
  for (int a = 0; a < 3; ++a) {
    if (shape[a] <= 0) return set_error(LBM_ERR_SHAPE, "lbm_tiles_build: shape[%d] = %d", a, shape[a]);
    n[a] = shape[a];
    if (((periodic >> a) & 1u) && n[a] % tile[a])
      return set_error(LBM_ERR_SHAPE, "lbm_tiles_build: periodic axis %d of size %lld is not a multiple of %d", a,
                       (long long)n[a], tile[a]);
    np[a] = (n[a] + tile[a] - 1) / tile[a] * tile[a];
    T[a] = np[a] / tile[a];
  }
  const int64_t ntn = (int64_t)tile[0] * tile[1] * tile[2];
  const int W = (int)(ntn / 64);
  const int64_t Ttot = T[0] * T[1] * T[2];
  if (Ttot > INT32_MAX) return set_error(LBM_ERR_SHAPE, "lbm_tiles_build: %lld tiles exceed int32", (long long)Ttot);

  lbm_tiles *t = new (std::nothrow) lbm_tiles();
  if (!t) return set_error(LBM_ERR_NOMEM, "lbm_tiles_build: out of host memory");
  try {
    std::vector<uint64_t> all((size_t)(Ttot * W), 0ull);
    // pass 1: per-tile fluid bits for every tile
    for (int64_t z = 0; z < n[2]; ++z) {
      const int64_t tz = z / tile[2], lz = z % tile[2];
      for (int64_t y = 0; y < n[1]; ++y) {
        const int64_t ty = y / tile[1], ly = y % tile[1];
        const uint8_t *row = solid + (z * n[1] + y) * n[0];
        for (int64_t x = 0; x < n[0]; ++x) {
          if (row[x]) continue;
          const int64_t tx = x / tile[0], lx = x % tile[0];
          const int64_t tid = (tz * T[1] + ty) * T[0] + tx;
          const int64_t l = lx + tile[0] * (ly + tile[1] * lz);
          all[(size_t)(tid * W + l / 64)] |= 1ull << (l % 64);
        }
      }
    }
    // pass 2: compact non-empty tiles in row-major tile order (tx fastest)
    t->tile_map.assign((size_t)Ttot, -1);
    int64_t nft = 0, nf = 0;
    for (int64_t tid = 0; tid < Ttot; ++tid) {
      bool any = false;
      for (int w = 0; w < W; ++w) any |= all[(size_t)(tid * W + w)] != 0;
      if (!any) continue;
      t->tile_map[(size_t)tid] = (int32_t)nft;
      t->coord.push_back((int32_t)(tid % T[0]));
      t->coord.push_back((int32_t)((tid / T[0]) % T[1]));
      t->coord.push_back((int32_t)(tid / (T[0] * T[1])));
      for (int w = 0; w < W; ++w) {
        uint64_t v = all[(size_t)(tid * W + w)];
        t->fluid.push_back(v);
        nf += __builtin_popcountll(v);
      }
      ++nft;
    }
    // neighbour rows
    t->nbr.resize((size_t)(nft * 27));
    for (int64_t k = 0; k < nft; ++k) {
      const int64_t c[3] = {t->coord[3 * k], t->coord[3 * k + 1], t->coord[3 * k + 2]};
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int d[3] = {dx, dy, dz};
            int64_t p[3];
            bool inside = true;
            for (int a = 0; a < 3; ++a) {
              p[a] = c[a] + d[a];
              if (p[a] < 0 || p[a] >= T[a]) {
                if ((periodic >> a) & 1u)
                  p[a] = (p[a] + T[a]) % T[a];
                else
                  inside = false;
              }
            }
            const int slot = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
            t->nbr[(size_t)(k * 27 + slot)] =
                inside ? t->tile_map[(size_t)((p[2] * T[1] + p[1]) * T[0] + p[0])] : -1;
          }
    }
    std::memcpy(t->tile, tile, sizeof t->tile);
    t->words = W;
    lbm::Sample s{};
    for (int a = 0; a < 3; ++a) {
      s.shape[a] = (int32_t)n[a];
      s.grid[a] = (int32_t)np[a];
      s.tgrid[a] = (int32_t)T[a];
    }
    s.periodic = periodic;
    s.tile0 = 0;
    s.n_ftiles = nft;
    s.map0 = 0;
    s.dense0 = 0;
    s.n_nodes = n[0] * n[1] * n[2];
    s.n_fluid = nf;
    t->samples.push_back(s);
    t->sample_of.assign((size_t)nft, 0);
    t->n_tiles = Ttot;
    t->n_ftiles = nft;
    t->n_fluid = nf;
    t->n_nodes = s.n_nodes;
  } catch (const std::bad_alloc &) {
    delete t;
    return set_error(LBM_ERR_NOMEM, "lbm_tiles_build: out of host memory");
  }
  *out = t;
  return LBM_OK;
}

extern "C" int lbm_tiles_info(const lbm_tiles *t, lbm_tiles_info_t *out) {
  if (!t || !out) return set_error(LBM_ERR_ARG, "lbm_tiles_info: NULL argument");
  std::memset(out, 0, sizeof *out);
  const lbm::Sample &s0 = t->samples.front();
  for (int a = 0; a < 3; ++a) {
    out->shape[a] = s0.shape[a];
    out->grid[a] = s0.grid[a];
    out->tile[a] = t->tile[a];
    out->tgrid[a] = s0.tgrid[a];
  }
  out->periodic = s0.periodic;
  out->words = t->words;
  out->n_samples = (int32_t)t->samples.size();
  out->n_tiles = t->n_tiles;
  out->n_ftiles = t->n_ftiles;
  out->n_fluid = t->n_fluid;
  out->n_nodes = t->n_nodes;
  out->phi = t->n_nodes ? (double)t->n_fluid / (double)t->n_nodes : 0.0;
  const double ntn = (double)t->tile[0] * t->tile[1] * t->tile[2];
  out->phi_t = t->n_ftiles ? (double)t->n_fluid / ((double)t->n_ftiles * ntn) : 0.0;
  out->tiles_ratio = t->n_ftiles ? (double)t->n_tiles / (double)t->n_ftiles : 0.0;
  // alpha_M (Sec. 3.1.1.2): faces of non-empty tiles across which the
  // neighbour tile is non-empty, over all faces of non-empty tiles; the faces
  // counted are those of the axes along which the lattice has more than one
  // node (two per axis)
  int64_t faces = 0, shared = 0;
  for (const lbm::Sample &S : t->samples) {
    for (int a = 0; a < 3; ++a) {
      if (S.grid[a] <= 1) continue;
      const int step = a == 0 ? 1 : a == 1 ? 3 : 9;
      for (int64_t k = S.tile0; k < S.tile0 + S.n_ftiles; ++k) {
        shared += (t->nbr[(size_t)(k * 27 + 13 - step)] >= 0) + (t->nbr[(size_t)(k * 27 + 13 + step)] >= 0);
        faces += 2;
      }
    }
  }
  out->alpha_m = faces ? (double)shared / (double)faces : 0.0;
  return LBM_OK;
}

extern "C" int lbm_tiles_export(const lbm_tiles *t, int32_t *tile_map, int32_t *tile_coord, int32_t *nbr,
                                uint64_t *fluid) {
  if (!t) return set_error(LBM_ERR_ARG, "lbm_tiles_export: NULL tiles");
  if (tile_map) std::memcpy(tile_map, t->tile_map.data(), t->tile_map.size() * sizeof(int32_t));
  if (tile_coord) std::memcpy(tile_coord, t->coord.data(), t->coord.size() * sizeof(int32_t));
  if (nbr) std::memcpy(nbr, t->nbr.data(), t->nbr.size() * sizeof(int32_t));
  if (fluid) std::memcpy(fluid, t->fluid.data(), t->fluid.size() * sizeof(uint64_t));
  return LBM_OK;
}

extern "C" int lbm_tiles_concat(const lbm_tiles *const *parts, int32_t k, lbm_tiles **out) {
  if (!parts || !out || k <= 0) return set_error(LBM_ERR_ARG, "lbm_tiles_concat: bad arguments");
  *out = nullptr;
  for (int32_t i = 0; i < k; ++i) {
    if (!parts[i]) return set_error(LBM_ERR_ARG, "lbm_tiles_concat: part %d is NULL", i);
    if (std::memcmp(parts[i]->tile, parts[0]->tile, sizeof parts[0]->tile))
      return set_error(LBM_ERR_ARG, "lbm_tiles_concat: part %d has a different tile shape", i);
  }
  lbm_tiles *t = new (std::nothrow) lbm_tiles();
  if (!t) return set_error(LBM_ERR_NOMEM, "lbm_tiles_concat: out of host memory");
  try {
    std::memcpy(t->tile, parts[0]->tile, sizeof t->tile);
    t->words = parts[0]->words;
    for (int32_t i = 0; i < k; ++i) {
      const lbm_tiles *p = parts[i];
      const int64_t toff = t->n_ftiles, moff = (int64_t)t->tile_map.size(), doff = t->n_nodes;
      for (const lbm::Sample &s : p->samples) {
        lbm::Sample c = s;
        c.tile0 += toff;
        c.map0 += moff;
        c.dense0 += doff;
        t->samples.push_back(c);
      }
      const int32_t soff = (int32_t)(t->samples.size() - p->samples.size());
      for (int32_t v : p->tile_map) t->tile_map.push_back(v < 0 ? -1 : (int32_t)(v + toff));
      t->coord.insert(t->coord.end(), p->coord.begin(), p->coord.end());
      for (int32_t v : p->nbr) t->nbr.push_back(v < 0 ? -1 : (int32_t)(v + toff));
      t->fluid.insert(t->fluid.end(), p->fluid.begin(), p->fluid.end());
      for (int32_t v : p->sample_of) t->sample_of.push_back(v + soff);
      t->n_tiles += p->n_tiles;
      t->n_ftiles += p->n_ftiles;
      t->n_fluid += p->n_fluid;
      t->n_nodes += p->n_nodes;
    }
    if (t->n_ftiles > INT32_MAX) {
      delete t;
      return set_error(LBM_ERR_SHAPE, "lbm_tiles_concat: too many tiles");
    }
  } catch (const std::bad_alloc &) {
    delete t;
    return set_error(LBM_ERR_NOMEM, "lbm_tiles_concat: out of host memory");
  }
  *out = t;
  return LBM_OK;
}

extern "C" void lbm_tiles_free(lbm_tiles *t) { delete t; }

extern "C" const char *lbm_last_error(void) { return lbm::last_error(); }

extern "C" const char *lbm_strerror(int code) {
  switch (code) {
    case LBM_OK: return "ok";
    case LBM_ERR_ARG: return "invalid argument";
    case LBM_ERR_SHAPE: return "invalid shape";
    case LBM_ERR_UNSUPPORTED: return "unsupported configuration";
    case LBM_ERR_HIP: return "HIP runtime error";
    case LBM_ERR_NONFINITE: return "non-finite value";
    case LBM_ERR_STATE: return "invalid call order";
    case LBM_ERR_NOMEM: return "out of memory";
    default: return "unknown error";
  }
}
