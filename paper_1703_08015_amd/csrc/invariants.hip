// Projection of a starting state onto the invariants of a start from rest:
// mass per lattice-connected component and, per axis k, the staggered
// momentum sum (-1)^{x_k} rho u_k per component of the c_k != 0 links.
//
// Four launches on the caller's stream: clear the per-component sums, sum
// (rho, 1) per component, rescale rho, sum ((-1)^{x_k} rho u_k, rho) per
// axis component, subtract the staggered mean.  Per-component sums use
// wave-aggregated FP64 atomics: the lanes of a wave that share a label are
// reduced with cross-lane shuffles and one lane adds the total, so a giant
// component costs one atomic per wave rather than one per node.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

using lbm::set_error;

namespace {

constexpr int kBlock = 256;

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

__device__ inline double parity_sign(int64_t i, int axis, int32_t nx, int32_t ny) {
  int64_t coord = axis == 0 ? i % nx : axis == 1 ? (i / nx) % ny : i / ((int64_t)nx * ny);
  return (coord & 1) ? -1.0 : 1.0;
}

__global__ void __launch_bounds__(kBlock) k_clear(double *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = 0.0;
}

// Labels outside [0, count) are treated as solid: a bad label array leaves
// its nodes untouched instead of adding out of bounds.
__device__ inline int checked(int32_t label, int32_t count) { return label < count ? label : -1; }

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

struct AxisSums {
  double *acc[3];     // per-axis (S, M) pairs
  int32_t count[3];   // components per axis
};

__global__ void __launch_bounds__(kBlock) k_staggered(int64_t n, int dims, int32_t nx, int32_t ny, const int32_t *lab,
                                                      const double *rho, const double *u, AxisSums sums) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  const bool in = i < n;
  for (int k = 0; k < dims; ++k) {
    int L = -1;
    double s = 0.0, m = 0.0;
    if (in) {
      L = checked(lab[(int64_t)(1 + k) * n + i], sums.count[k]);
      if (L >= 0) {
        m = rho[i];
        s = parity_sign(i, k, nx, ny) * m * u[(int64_t)k * n + i];
      }
    }
    wave_add2(sums.acc[k], L, s, m);
  }
}

__global__ void __launch_bounds__(kBlock) k_unstagger(int64_t n, int dims, int32_t nx, int32_t ny,
                                                      const int32_t *lab, AxisSums sums, double *u) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < dims; ++k) {
    const int L = checked(lab[(int64_t)(1 + k) * n + i], sums.count[k]);
    if (L < 0) continue;
    const double *a = sums.acc[k] + 2 * (int64_t)L;
    u[(int64_t)k * n + i] -= parity_sign(i, k, nx, ny) * (a[0] / a[1]);
  }
}

}  // namespace

extern "C" int lbm_project_invariants(int32_t q, const int32_t shape[3], const int32_t *labels, const int32_t *counts,
                                      double rho0, double *rho, double *u, double *scratch, void *stream) {
  if (!shape || !labels || !counts || !rho || !u || !scratch)
    return set_error(LBM_ERR_ARG, "lbm_project_invariants: NULL argument");
  if (q != 9 && q != 19) return set_error(LBM_ERR_UNSUPPORTED, "lbm_project_invariants: q = %d", q);
  const int dims = q == 9 ? 2 : 3;
  if (shape[0] <= 0 || shape[1] <= 0 || shape[2] <= 0 || (q == 9 && shape[2] != 1))
    return set_error(LBM_ERR_ARG, "lbm_project_invariants: shape %d x %d x %d for q = %d", shape[0], shape[1],
                     shape[2], q);
  if (!(rho0 > 0.0) || rho0 != rho0 || rho0 > 1e300)
    return set_error(LBM_ERR_ARG, "lbm_project_invariants: rho0 = %g", rho0);
  const int64_t n = (int64_t)shape[0] * shape[1] * shape[2];
  int64_t total = 0;
  for (int k = 0; k <= dims; ++k) {
    if (counts[k] < 0) return set_error(LBM_ERR_ARG, "lbm_project_invariants: counts[%d] = %d", k, counts[k]);
    if (counts[k] > n) return set_error(LBM_ERR_ARG, "lbm_project_invariants: counts[%d] = %d > %lld nodes", k,
                                        counts[k], (long long)n);
    total += counts[k];
  }
  if (counts[0] == 0) return LBM_OK;  // no non-solid node
  hipStream_t s = (hipStream_t)stream;
  const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
  const unsigned clear_grid = (unsigned)std::min<int64_t>((2 * total + kBlock - 1) / kBlock, 4096);
  AxisSums sums{};
  int64_t off = 2 * (int64_t)counts[0];
  for (int k = 0; k < dims; ++k) {
    sums.acc[k] = scratch + off;
    sums.count[k] = counts[1 + k];
    off += 2 * (int64_t)counts[1 + k];
  }
  hipLaunchKernelGGL(k_clear, dim3(clear_grid), dim3(kBlock), 0, s, scratch, 2 * total);
  hipLaunchKernelGGL(k_mass, dim3(grid), dim3(kBlock), 0, s, n, labels, counts[0], (const double *)rho, scratch);
  hipLaunchKernelGGL(k_rescale, dim3(grid), dim3(kBlock), 0, s, n, labels, counts[0], (const double *)scratch, rho0, rho);
  hipLaunchKernelGGL(k_staggered, dim3(grid), dim3(kBlock), 0, s, n, dims, shape[0], shape[1], labels,
                     (const double *)rho, (const double *)u, sums);
  hipLaunchKernelGGL(k_unstagger, dim3(grid), dim3(kBlock), 0, s, n, dims, shape[0], shape[1], labels, sums, u);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(LBM_ERR_HIP, "lbm_project_invariants: %s", hipGetErrorString(e));
  return LBM_OK;
}
