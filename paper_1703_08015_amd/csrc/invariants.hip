// Projection of a starting state onto the invariants of a start from rest.
//
// Mass: rho is rescaled per lattice-connected component so that it holds
// rho0 per node.  Staggered momentum: the invariants are the functionals
// sum_x beta(x).j(x) with beta in the null space of the link operator
// (A beta)_link = c.beta(x+c) + c.beta(x); the operator
//   (T j)(x) = 3 sum_{i: x + c_i fluid} w_i c_i [c_i.(j(x) + j(x + c_i))] / 2
// equals (3/2) A^T W A, so its range is orthogonal to all of them, and the
// Richardson sweeps j <- j + T(rho u - j) from j = 0 give a momentum field
// with none of them while approaching rho u (T is the identity on smooth
// fields in the bulk, with eigenvalues in [0, 1]).
//
// Launches on the caller's stream: clear the per-component sums, sum
// (rho, 1) per component, rescale rho, one stencil launch per sweep
// (ping-pong buffers in the scratch), then u = j / rho.  Per-component sums
// use wave-aggregated FP64 atomics: the lanes of a wave that share a label
// are reduced with cross-lane shuffles and one lane adds the total, so a
// giant component costs one atomic per wave rather than one per node.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "device.h"
#include "internal.h"

using lbm::set_error;

namespace {

constexpr int kBlock = 256;
constexpr int kMaxIterations = 1000;

// Add (a, b) of every lane to acc[2*label], acc[2*label + 1]; lanes with a
// negative label add nothing.  Every lane of the wave must call it.
__device__ inline void wave_add2(double *acc, int label, double a, double b) {
  unsigned long long pending = __ballot(label >= 0);
  const int lane = __lane_id();
  while (pending) {
    const int leader = __ffsll(pending) - 1;
    const int L = __shfl(label, leader);
    const bool mine = label == L;
    double x = mine ? a : 0.0, y = mine ? b : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      x += __shfl_xor(x, off);
      y += __shfl_xor(y, off);
    }
    if (lane == leader) {
      unsafeAtomicAdd(acc + 2 * (int64_t)L, x);
      unsafeAtomicAdd(acc + 2 * (int64_t)L + 1, y);
    }
    pending &= ~__ballot(mine);
  }
}

// Labels outside [0, count) are treated as solid: a bad label array leaves
// its nodes untouched instead of adding out of bounds.
__device__ inline int checked(int32_t label, int32_t count) { return label < count ? label : -1; }

__global__ void __launch_bounds__(kBlock) k_clear(double *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = 0.0;
}

__global__ void __launch_bounds__(kBlock) k_mass(int64_t n, const int32_t *lab, int32_t count, const double *rho,
                                                 double *acc) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  int L = -1;
  double r = 0.0;
  if (i < n) {
    L = checked(lab[i], count);
    if (L >= 0) r = rho[i];
  }
  wave_add2(acc, L, r, 1.0);
}

__global__ void __launch_bounds__(kBlock) k_rescale(int64_t n, const int32_t *lab, int32_t count, const double *acc,
                                                    double rho0, double *rho) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= n) return;
  const int L = checked(lab[i], count);
  if (L < 0) return;
  rho[i] = rho[i] * (rho0 * acc[2 * (int64_t)L + 1] / acc[2 * (int64_t)L]);
}

struct Lattice3 {
  int32_t nx, ny, nz;
  uint32_t periodic;
};

// j_out = j_in + T(rho u - j_in) on non-solid nodes (0 on solid ones); with
// j_in == nullptr the sweep starts from j = 0.
template <class L>
__global__ void __launch_bounds__(kBlock) k_link_sweep(int64_t n, Lattice3 g, const int32_t *lab, int32_t count,
                                                       const double *rho, const double *u, const double *j_in,
                                                       double *j_out) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= n) return;
  if (checked(lab[i], count) < 0) {
    j_out[i] = j_out[n + i] = j_out[2 * n + i] = 0.0;
    return;
  }
  const int x = (int)(i % g.nx), y = (int)((i / g.nx) % g.ny), z = (int)(i / ((int64_t)g.nx * g.ny));
  auto residual = [&](int64_t p, int k) {
    const double j = j_in ? j_in[k * n + p] : 0.0;
    return rho[p] * u[k * n + p] - j;
  };
  const double r0[3] = {residual(i, 0), residual(i, 1), residual(i, 2)};
  double acc[3] = {0.0, 0.0, 0.0};
  lbm::static_for<L::Q>([&](auto d) {
    constexpr int cx = L::C[d][0], cy = L::C[d][1], cz = L::C[d][2];
    if constexpr (cx != 0 || cy != 0 || cz != 0) {
      int tx = x + cx, ty = y + cy, tz = z + cz;
      bool inside = true;
      if (tx < 0 || tx >= g.nx) {
        inside &= (g.periodic & 1u) != 0;
        tx = tx < 0 ? tx + g.nx : tx - g.nx;
      }
      if (ty < 0 || ty >= g.ny) {
        inside &= (g.periodic & 2u) != 0;
        ty = ty < 0 ? ty + g.ny : ty - g.ny;
      }
      if (tz < 0 || tz >= g.nz) {
        inside &= (g.periodic & 4u) != 0;
        tz = tz < 0 ? tz + g.nz : tz - g.nz;
      }
      if (inside) {
        const int64_t t = (int64_t)tx + (int64_t)g.nx * ((int64_t)ty + (int64_t)g.ny * tz);
        if (checked(lab[t], count) >= 0) {
          double s = 0.0;
          if constexpr (cx != 0) s += cx * (r0[0] + residual(t, 0));
          if constexpr (cy != 0) s += cy * (r0[1] + residual(t, 1));
          if constexpr (cz != 0) s += cz * (r0[2] + residual(t, 2));
          s *= 1.5 * L::Wt[d];
          if constexpr (cx != 0) acc[0] += cx * s;
          if constexpr (cy != 0) acc[1] += cy * s;
          if constexpr (cz != 0) acc[2] += cz * s;
        }
      }
    }
  });
  for (int k = 0; k < 3; ++k) j_out[k * n + i] = (j_in ? j_in[k * n + i] : 0.0) + acc[k];
}

__global__ void __launch_bounds__(kBlock) k_velocity(int64_t n, const int32_t *lab, int32_t count, const double *rho,
                                                     const double *j, double *u) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= n || checked(lab[i], count) < 0) return;
  const double r = rho[i];
  for (int k = 0; k < 3; ++k) u[k * n + i] = j[k * n + i] / r;
}

template <class L>
void launch_sweeps(int64_t n, Lattice3 g, const int32_t *labels, int32_t count, const double *rho, const double *u,
                   double *ja, double *jb, int iterations, hipStream_t s, const double **final_j) {
  const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
  const double *in = nullptr;
  double *out = ja;
  for (int it = 0; it < iterations; ++it) {
    hipLaunchKernelGGL(k_link_sweep<L>, dim3(grid), dim3(kBlock), 0, s, n, g, labels, count, rho, u, in, out);
    in = out;
    out = out == ja ? jb : ja;
  }
  *final_j = in;
}

}  // namespace

extern "C" int lbm_project_invariants(int32_t q, const int32_t shape[3], uint32_t periodic, const int32_t *labels,
                                      int32_t count, double rho0, int32_t iterations, double *rho, double *u,
                                      double *scratch, void *stream) {
  if (!shape || !labels || !rho || !u || !scratch)
    return set_error(LBM_ERR_ARG, "lbm_project_invariants: NULL argument");
  if (q != 9 && q != 19) return set_error(LBM_ERR_UNSUPPORTED, "lbm_project_invariants: q = %d", q);
  if (shape[0] <= 0 || shape[1] <= 0 || shape[2] <= 0 || (q == 9 && shape[2] != 1))
    return set_error(LBM_ERR_ARG, "lbm_project_invariants: shape %d x %d x %d for q = %d", shape[0], shape[1],
                     shape[2], q);
  if (periodic > 7u) return set_error(LBM_ERR_ARG, "lbm_project_invariants: periodic bits %u", periodic);
  if (!(rho0 > 0.0) || rho0 > 1e300) return set_error(LBM_ERR_ARG, "lbm_project_invariants: rho0 = %g", rho0);
  if (iterations < 1 || iterations > kMaxIterations)
    return set_error(LBM_ERR_ARG, "lbm_project_invariants: iterations = %d (1..%d)", iterations, kMaxIterations);
  const int64_t n = (int64_t)shape[0] * shape[1] * shape[2];
  if (count < 0 || count > n)
    return set_error(LBM_ERR_ARG, "lbm_project_invariants: count = %d for %lld nodes", count, (long long)n);
  if (count == 0) return LBM_OK;  // no non-solid node
  hipStream_t s = (hipStream_t)stream;
  const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
  const int64_t sums = 2 * (int64_t)count;
  const unsigned clear_grid = (unsigned)std::min<int64_t>((sums + kBlock - 1) / kBlock, 4096);
  double *acc = scratch;
  double *ja = scratch + sums, *jb = ja + 3 * n;
  hipLaunchKernelGGL(k_clear, dim3(clear_grid), dim3(kBlock), 0, s, acc, sums);
  hipLaunchKernelGGL(k_mass, dim3(grid), dim3(kBlock), 0, s, n, labels, count, (const double *)rho, acc);
  hipLaunchKernelGGL(k_rescale, dim3(grid), dim3(kBlock), 0, s, n, labels, count, (const double *)acc, rho0, rho);
  const Lattice3 g{shape[0], shape[1], shape[2], periodic};
  const double *j = nullptr;
  if (q == 19)
    launch_sweeps<lbm::D3Q19>(n, g, labels, count, rho, u, ja, jb, iterations, s, &j);
  else
    launch_sweeps<lbm::D2Q9>(n, g, labels, count, rho, u, ja, jb, iterations, s, &j);
  hipLaunchKernelGGL(k_velocity, dim3(grid), dim3(kBlock), 0, s, n, labels, count, (const double *)rho, j, u);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(LBM_ERR_HIP, "lbm_project_invariants: %s", hipGetErrorString(e));
  return LBM_OK;
}

// ---- connected components on the device ---------------------------------------
// The same labels as the host lbm_components, for a warm start that must
// not wait for the host.  Lock-free union-find over the links: every
// pointer goes from a node to a node of smaller index, a union hooks the
// larger of two roots under the smaller with a compare-and-swap (retrying
// from the new parent if the root moved meanwhile), and finds halve their
// paths.  Because every parent index is smaller than its node's, every loop
// ends: a find walks strictly decreasing indices and a failed hook lowers
// the larger root.  The root of a component is then its smallest node, so
// numbering roots in scan order (an exclusive prefix sum of root flags)
// reproduces the host's numbering by first appearance.
namespace {

constexpr int kScanBlock = 1024;  // threads of the scan kernels
constexpr int kScanItems = 4;     // items per thread

__device__ __forceinline__ int32_t ld_parent(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t cc_find(int32_t *parent, int32_t v) {
  while (true) {
    const int32_t p = ld_parent(parent + v);
    if (p == v) return v;
    const int32_t gp = ld_parent(parent + p);
    if (gp == p) return p;
    __hip_atomic_store(parent + v, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // an ancestor of v
    v = gp;
  }
}

__global__ void __launch_bounds__(kBlock) k_cc_init(int64_t n, const uint8_t *solid, int32_t *parent) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += (int64_t)gridDim.x * kBlock)
    parent[e] = solid[e] ? -1 : (int32_t)e;
}

struct CcGrid {
  int nx, ny, nz;
};

// One thread per node: union with the non-solid node one link away, for one
// link of each opposite pair (only links with c_axis != 0 when axis >= 0).
template <class L>
__global__ void __launch_bounds__(kBlock) k_cc_union(CcGrid g, uint32_t periodic, int axis, const uint8_t *solid,
                                                     int32_t *parent) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n || solid[e]) return;
  const int x = (int)(e % g.nx), y = (int)((e / g.nx) % g.ny), z = (int)(e / ((int64_t)g.nx * g.ny));
  lbm::static_for<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = L::C[i][0], cy = L::C[i][1], cz = L::C[i][2];
    if constexpr ((cx != 0 || cy != 0 || cz != 0) && i < L::Opp[i]) {
      const int c[3] = {cx, cy, cz};
      if (axis >= 0 && c[axis] == 0) return;
      int t[3] = {x + cx, y + cy, z + cz};
      const int ext[3] = {g.nx, g.ny, g.nz};
      for (int a = 0; a < 3; ++a) {
        if (t[a] >= 0 && t[a] < ext[a]) continue;
        if (!((periodic >> a) & 1u)) return;
        t[a] = t[a] < 0 ? t[a] + ext[a] : t[a] - ext[a];
      }
      const int64_t f = (int64_t)t[0] + (int64_t)g.nx * ((int64_t)t[1] + (int64_t)g.ny * t[2]);
      if (solid[f]) return;
      int32_t a = cc_find(parent, (int32_t)e), b = cc_find(parent, (int32_t)f);
      while (a != b) {
        if (a > b) {
          const int32_t s = a;
          a = b;
          b = s;
        }
        const int32_t old = atomicCAS(parent + b, b, a);
        if (old == b) break;  // b now hangs under a
        b = cc_find(parent, old);
        a = cc_find(parent, a);
      }
    }
  });
}

// parent <- root; flag = 1 on roots (in the scan buffer).  The walk to the
// root only reads: the single write per node is its root, so a concurrent
// walk through that node sees an ancestor either way, and every node ends
// holding its root.
__global__ void __launch_bounds__(kBlock) k_cc_flatten(int64_t n, int32_t *parent, int32_t *flag) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += (int64_t)gridDim.x * kBlock) {
    const int32_t p = parent[e];
    if (p < 0) {
      flag[e] = 0;
      continue;
    }
    int32_t r = (int32_t)e;
    for (int32_t up = p; up != r; up = ld_parent(parent + up)) r = up;
    flag[e] = r == (int32_t)e;
    __hip_atomic_store(parent + e, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Exclusive prefix sum of v[0, n) in place, kScanBlock * kScanItems items per
// block; the block totals go to sums[blockIdx.x].
__global__ void __launch_bounds__(kScanBlock) k_scan_block(int64_t n, int32_t *v, int32_t *sums) {
  __shared__ int32_t s[kScanBlock];
  const int64_t base = ((int64_t)blockIdx.x * kScanBlock + threadIdx.x) * kScanItems;
  int32_t item[kScanItems], run = 0;
  for (int k = 0; k < kScanItems; ++k) {
    item[k] = base + k < n ? v[base + k] : 0;
    run += item[k];
  }
  s[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {  // inclusive Hillis-Steele scan of the thread totals
    const int32_t t = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  int32_t acc = s[threadIdx.x] - run;
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) v[base + k] = acc;
    acc += item[k];
  }
  if (threadIdx.x == kScanBlock - 1) sums[blockIdx.x] = s[threadIdx.x];
}

// Exclusive scan of the block totals (one block, any count); total to sums[nb].
__global__ void __launch_bounds__(kScanBlock) k_scan_sums(int64_t nb, int32_t *sums) {
  __shared__ int32_t s[kScanBlock];
  int32_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kScanBlock) {
    const int64_t b = b0 + threadIdx.x;
    const int32_t x = b < nb ? sums[b] : 0;
    s[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
      const int32_t t = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    if (b < nb) sums[b] = carry + s[threadIdx.x] - x;
    const int32_t total = s[kScanBlock - 1];
    __syncthreads();
    carry += total;
  }
  if (threadIdx.x == 0) sums[nb] = carry;
}

// labels = rank of the node's root among the roots (the root's flag slot
// holds it once offset by its block's total); -1 on solid nodes
__global__ void __launch_bounds__(kBlock) k_cc_label(int64_t n, const int32_t *rank, const int32_t *sums,
                                                     int32_t *parent_to_label) {
  constexpr int64_t per = (int64_t)kScanBlock * kScanItems;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += (int64_t)gridDim.x * kBlock) {
    const int32_t r = parent_to_label[e];
    parent_to_label[e] = r < 0 ? -1 : rank[r] + sums[r / per];
  }
}

unsigned cc_grid(int64_t n) {
  const int64_t b = (n + kBlock - 1) / kBlock;
  return (unsigned)(b < 16384 ? (b > 0 ? b : 1) : 16384);
}

}  // namespace

extern "C" int64_t lbm_components_device_scratch(const int32_t shape[3]) {
  if (!shape || shape[0] <= 0 || shape[1] <= 0 || shape[2] <= 0) return -1;
  const int64_t n = (int64_t)shape[0] * shape[1] * shape[2];
  const int64_t per = (int64_t)kScanBlock * kScanItems;
  return n + (n + per - 1) / per + 1;
}

namespace {

// The labelling behind both device entry points; scratch holds
// lbm_components_device_scratch(shape) int32 entries, every one written
// before it is read.
int components_device(const char *who, int32_t q, const uint8_t *solid, const int32_t shape[3], uint32_t periodic,
                      int32_t axis, int32_t *labels, int32_t *count, int32_t *scratch, hipStream_t s) {
  const int64_t n = (int64_t)shape[0] * shape[1] * shape[2];
  const CcGrid g{shape[0], shape[1], shape[2]};
  const int64_t per = (int64_t)kScanBlock * kScanItems, nb = (n + per - 1) / per;
  int32_t *flag = scratch, *sums = scratch + n;
  hipLaunchKernelGGL(k_cc_init, dim3(cc_grid(n)), dim3(kBlock), 0, s, n, solid, labels);
  const unsigned all = (unsigned)((n + kBlock - 1) / kBlock);
  if (q == 19)
    hipLaunchKernelGGL(k_cc_union<lbm::D3Q19>, dim3(all), dim3(kBlock), 0, s, g, periodic, axis, solid, labels);
  else
    hipLaunchKernelGGL(k_cc_union<lbm::D2Q9>, dim3(all), dim3(kBlock), 0, s, g, periodic, axis, solid, labels);
  hipLaunchKernelGGL(k_cc_flatten, dim3(cc_grid(n)), dim3(kBlock), 0, s, n, labels, flag);
  hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(kScanBlock), 0, s, n, flag, sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, s, nb, sums);
  hipLaunchKernelGGL(k_cc_label, dim3(cc_grid(n)), dim3(kBlock), 0, s, n, flag, sums, labels);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(count, sums + nb, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return set_error(LBM_ERR_HIP, "%s: %s", who, hipGetErrorString(e));
  return LBM_OK;
}

// Argument checks shared by both device entry points.
int components_device_args(const char *who, int32_t q, const uint8_t *solid, const int32_t shape[3],
                           uint32_t periodic, int32_t axis, const int32_t *labels, const int32_t *count) {
  if (!solid || !shape || !labels || !count) return set_error(LBM_ERR_ARG, "%s: NULL argument", who);
  if (q != 9 && q != 19) return set_error(LBM_ERR_UNSUPPORTED, "%s: q = %d", who, q);
  if (shape[0] <= 0 || shape[1] <= 0 || shape[2] <= 0)
    return set_error(LBM_ERR_ARG, "%s: shape %d x %d x %d", who, shape[0], shape[1], shape[2]);
  if (q == 9 && shape[2] != 1) return set_error(LBM_ERR_ARG, "%s: D2Q9 needs shape[2] = 1", who);
  if (periodic > 7u) return set_error(LBM_ERR_ARG, "%s: periodic bits %u", who, periodic);
  if (axis < -1 || axis >= (q == 9 ? 2 : 3)) return set_error(LBM_ERR_ARG, "%s: axis %d for q = %d", who, axis, q);
  const int64_t n = (int64_t)shape[0] * shape[1] * shape[2];
  if (n > INT32_MAX) return set_error(LBM_ERR_ARG, "%s: %lld nodes exceed int32 labels", who, (long long)n);
  return LBM_OK;
}

// Fixed scratch of lbm_components_device_noalloc: one copy per GPU, held
// until the process ends.  Host code never passes this name to a kernel (on
// the host it is only a stand-in for the symbol); it uses the device address
// hipGetSymbolAddress returns for the current device.
constexpr int64_t kNoAllocEntries = int64_t(1) << 22;  // int32 entries, 16 MiB
static __device__ __align__(256) int32_t cc_noalloc_scratch[kNoAllocEntries];

constexpr int kMaxDevices = 64;

// Device address of cc_noalloc_scratch on the current device, looked up
// once per device (with that device current) and kept.
int noalloc_scratch(const char *who, int32_t **out) {
  static std::mutex mu;
  static int32_t *addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(LBM_ERR_HIP, "%s: %s", who, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_error(LBM_ERR_UNSUPPORTED, "%s: device %d", who, dev);
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(cc_noalloc_scratch));
    if (e != hipSuccess || !p)
      return set_error(LBM_ERR_HIP, "%s: scratch address: %s", who, hipGetErrorString(e));
    addr[dev] = static_cast<int32_t *>(p);
  }
  *out = addr[dev];
  return LBM_OK;
}

}  // namespace

extern "C" int lbm_components_device(int32_t q, const uint8_t *solid, const int32_t shape[3], uint32_t periodic,
                                     int32_t axis, int32_t *labels, int32_t *count, int32_t *scratch,
                                     void *stream) {
  const char *who = "lbm_components_device";
  if (!scratch) return set_error(LBM_ERR_ARG, "%s: NULL argument", who);
  const int r = components_device_args(who, q, solid, shape, periodic, axis, labels, count);
  if (r != LBM_OK) return r;
  return components_device(who, q, solid, shape, periodic, axis, labels, count, scratch,
                           static_cast<hipStream_t>(stream));
}

extern "C" int64_t lbm_components_noalloc_max_scratch(void) { return kNoAllocEntries; }

extern "C" int lbm_components_device_noalloc(int32_t q, const uint8_t *solid, const int32_t shape[3],
                                             uint32_t periodic, int32_t axis, int32_t *labels, int32_t *count,
                                             void *stream) {
  const char *who = "lbm_components_device_noalloc";
  const int r = components_device_args(who, q, solid, shape, periodic, axis, labels, count);
  if (r != LBM_OK) return r;
  const int64_t need = lbm_components_device_scratch(shape);
  if (need > kNoAllocEntries)
    return set_error(LBM_ERR_ARG, "%s: %d x %d x %d needs %lld scratch entries, above the fixed %lld", who, shape[0],
                     shape[1], shape[2], (long long)need, (long long)kNoAllocEntries);
  int32_t *scratch = nullptr;
  const int e = noalloc_scratch(who, &scratch);
  if (e != LBM_OK) return e;
  return components_device(who, q, solid, shape, periodic, axis, labels, count, scratch,
                           static_cast<hipStream_t>(stream));
}
