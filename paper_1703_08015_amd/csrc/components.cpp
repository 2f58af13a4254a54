// Connected components of the non-solid nodes under lattice links (host).
//
// Union-find over the dense lattice: every non-solid node is joined to the
// non-solid node one link away for each link of the velocity set (one of
// each opposite pair), restricted to links with c_axis != 0 when an axis is
// given.  A periodic axis wraps; a non-periodic edge is a wall, exactly as
// propagation treats it.
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

using lbm::set_error;

namespace {

struct DisjointSets {
  std::vector<int32_t> parent;
  explicit DisjointSets(int64_t n) : parent(n) {
    for (int64_t i = 0; i < n; ++i) parent[i] = (int32_t)i;
  }
  int32_t find(int32_t a) {
    while (parent[a] != a) {
      parent[a] = parent[parent[a]];  // path halving
      a = parent[a];
    }
    return a;
  }
  void unite(int32_t a, int32_t b) {
    a = find(a);
    b = find(b);
    if (a == b) return;
    if (a < b)
      parent[b] = a;
    else
      parent[a] = b;
  }
};

}  // namespace

extern "C" int lbm_components(int32_t q, const uint8_t *solid, const int32_t shape[3], uint32_t periodic,
                              int32_t axis, int32_t *labels, int32_t *count) {
  if (!solid || !shape || !labels || !count) return set_error(LBM_ERR_ARG, "lbm_components: NULL argument");
  if (q != 9 && q != 19) return set_error(LBM_ERR_UNSUPPORTED, "lbm_components: q = %d", q);
  const int dims = q == 9 ? 2 : 3;
  const int64_t nx = shape[0], ny = shape[1], nz = shape[2];
  if (nx <= 0 || ny <= 0 || nz <= 0) return set_error(LBM_ERR_ARG, "lbm_components: shape %lld x %lld x %lld",
                                                      (long long)nx, (long long)ny, (long long)nz);
  if (q == 9 && nz != 1) return set_error(LBM_ERR_ARG, "lbm_components: D2Q9 needs shape[2] = 1");
  if (periodic > 7u) return set_error(LBM_ERR_ARG, "lbm_components: periodic bits %u", periodic);
  if (axis < -1 || axis >= dims) return set_error(LBM_ERR_ARG, "lbm_components: axis %d for q = %d", axis, q);
  const int64_t n = nx * ny * nz;
  if (n > INT32_MAX) return set_error(LBM_ERR_ARG, "lbm_components: %lld nodes exceed int32 labels", (long long)n);

  int32_t c[3 * 19], opp[19];
  double w[19];
  int rc = lbm_lattice(q, c, w, opp);
  if (rc) return rc;

  try {
    DisjointSets ds(n);
    const int64_t ext[3] = {nx, ny, nz};
    for (int i = 0; i < q; ++i) {
      const int *ci = c + 3 * i;
      if (!ci[0] && !ci[1] && !ci[2]) continue;
      if (i > opp[i]) continue;  // one link of each opposite pair
      if (axis >= 0 && ci[axis] == 0) continue;
      for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
          for (int64_t x = 0; x < nx; ++x) {
            const int64_t p = x + nx * (y + ny * z);
            if (solid[p]) continue;
            int64_t t[3] = {x + ci[0], y + ci[1], z + ci[2]};
            bool inside = true;
            for (int a = 0; a < 3; ++a) {
              if (t[a] >= 0 && t[a] < ext[a]) continue;
              if (!(periodic >> a & 1u)) {
                inside = false;
                break;
              }
              t[a] = (t[a] + ext[a]) % ext[a];
            }
            if (!inside) continue;
            const int64_t r = t[0] + nx * (t[1] + ny * t[2]);
            if (!solid[r]) ds.unite((int32_t)p, (int32_t)r);
          }
    }
    std::vector<int32_t> label_of_root(n, -1);
    int32_t next = 0;
    for (int64_t p = 0; p < n; ++p) {
      if (solid[p]) {
        labels[p] = -1;
        continue;
      }
      const int32_t root = ds.find((int32_t)p);
      if (label_of_root[root] < 0) label_of_root[root] = next++;
      labels[p] = label_of_root[root];
    }
    *count = next;
  } catch (const std::bad_alloc &) {
    return set_error(LBM_ERR_NOMEM, "lbm_components: host allocation of %lld nodes failed", (long long)n);
  }
  return LBM_OK;
}
