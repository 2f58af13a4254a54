// Internal host-side structures of liblbm (not part of the C ABI).
#pragma once

#include <cstdarg>
#include <cstdint>
#include <string>
#include <vector>

#include "lbm.h"

namespace lbm {

// One geometry of a (possibly concatenated) tiling.
struct Sample {
  int32_t shape[3];   // lattice as given (nx, ny, nz)
  int32_t grid[3];    // padded
  int32_t tgrid[3];   // tiles per axis
  uint32_t periodic;  // bit 0 x, bit 1 y, bit 2 z
  int64_t tile0;      // first global non-empty tile
  int64_t n_ftiles;   // non-empty tiles of this sample
  int64_t map0;       // first entry of this sample in tile_map
  int64_t dense0;     // first node of this sample in concatenated dense arrays
  int64_t n_nodes;    // nx*ny*nz
  int64_t n_fluid;    // non-solid nodes
};

}  // namespace lbm

struct lbm_tiles {
  int32_t tile[3] = {0, 0, 0};
  int32_t words = 0;                 // 64-bit mask words per tile
  std::vector<lbm::Sample> samples;  // one entry unless concatenated
  std::vector<int32_t> tile_map;     // per sample, T_total entries each
  std::vector<int32_t> coord;        // 3 per non-empty tile
  std::vector<int32_t> nbr;          // 27 per non-empty tile (global indices)
  std::vector<uint64_t> fluid;       // words per non-empty tile
  std::vector<int32_t> sample_of;    // sample index per non-empty tile
  int64_t n_tiles = 0, n_ftiles = 0, n_fluid = 0, n_nodes = 0;
};

namespace lbm {

// Thread-local error text behind lbm_last_error().
int set_error(int code, const char *fmt, ...);
const char *last_error();

}  // namespace lbm
