// Layer kernels of the warm-start U-Net (C ABI in lbm_nn.h), gfx950.
//
// All convolutions are gather-GEMMs on BF16 MFMA (v_mfma_f32_16x16x32_bf16,
// FP32 accumulation): GEMM rows are voxels, the reduction runs over
// (tap, input channel) and columns are output channels.  Lane l of a
// wavefront holds A[l%16][8(l/16)..+7], B[8(l/16)..+7][l%16] and the result
// C[4(l/16)..+3][l%16]; with channels-last activations the A operand of a row
// is one 16-byte load of 8 consecutive channels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <initializer_list>

#include "device.h"
#include "internal.h"
#include "lbm_nn.h"

namespace lbm {
namespace nn {
namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct Grid {
  int nx, ny, nz;
};

struct GemmArgs {
  Grid rows, in_grid, out_grid;
  int taps, cin, cout, ldx, ldy;
  int64_t M;  // GEMM rows
  const bf16 *x;
  const bf16 *w;
  const float *bias;
  void *y;
  const bf16 *gate;  // ReLU gate of a backward-data pass (NULL: none)
  int ldg, gate_ch;
};

// the derivative of a ReLU whose output is g: 1 where g > 0 (NaN: 0)
__device__ __forceinline__ bool gate_open(bf16 g) { return (float)g > 0.f; }

__device__ __forceinline__ int64_t vidx(int x, int y, int z, const Grid &g) {
  return (int64_t)x + (int64_t)g.nx * ((int64_t)y + (int64_t)g.ny * z);
}

// periodic wrap of a coordinate within one period of the grid: v in [-n, 2n)
__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// input voxel of GEMM row m for tap t
template <int SRC>
__device__ __forceinline__ int64_t src_voxel(int64_t m, int t, const Grid &rows, const Grid &in) {
  if constexpr (SRC == LBM_NN_IDENT) {
    return m;
  } else {
    const int x = (int)(m % rows.nx), y = (int)((m / rows.nx) % rows.ny), z = (int)(m / ((int64_t)rows.nx * rows.ny));
    if constexpr (SRC == LBM_NN_CONV3) {
      int sx = x + t % 3 - 1, sy = y + (t / 3) % 3 - 1, sz = z + t / 9 - 1;
      sx += sx < 0 ? in.nx : (sx >= in.nx ? -in.nx : 0);
      sy += sy < 0 ? in.ny : (sy >= in.ny ? -in.ny : 0);
      sz += sz < 0 ? in.nz : (sz >= in.nz ? -in.nz : 0);
      return vidx(sx, sy, sz, in);
    } else {  // GATHER2
      return vidx(2 * x + (t & 1), 2 * y + ((t >> 1) & 1), 2 * z + (t >> 2), in);
    }
  }
}

template <int DST>
__device__ __forceinline__ int64_t dst_voxel(int64_t m, int t, const Grid &rows, const Grid &out) {
  if constexpr (DST == LBM_NN_IDENT) {
    return m;
  } else {
    const int mi = (int)m;  // rows are checked to number fewer than 2^31
    const int x = mi % rows.nx, y = (mi / rows.nx) % rows.ny, z = mi / (rows.nx * rows.ny);
    return vidx(2 * x + (t & 1), 2 * y + ((t >> 1) & 1), 2 * z + (t >> 2), out);
  }
}

// ---- forward gather-GEMM ----------------------------------------------------
// Block: 4 wavefronts x 16*RF rows (RF 16-row fragments each; RF = 1 for
// grids too small to fill the device otherwise) x 16*NW columns.
// K runs over the flattened (tap, channel) index k = t*cin + c: cin is a
// multiple of 8, so each lane's 8-channel group lies inside one tap and
// gathers its own input row, and no K is padded per tap (the first layer's 8
// input channels fill whole 32-wide K steps).  Each K step's weight tile
// (16*NW columns x 32 k) is staged once per block in LDS, double-buffered, and
// read by all four wavefronts; the gathered input rows of the next K step are
// loaded while the current step's MFMAs run; a row's voxel coordinates are
// decoded once.
constexpr int kLdsK = 40;  // 32 k + 8 bf16 of padding per LDS row

template <int SRC>
__device__ __forceinline__ int64_t gather_row(int x, int y, int z, int64_t m, int t, const Grid &in) {
  if constexpr (SRC == LBM_NN_IDENT) {
    return m;
  } else if constexpr (SRC == LBM_NN_CONV3) {
    int sx = x + t % 3 - 1, sy = y + (t / 3) % 3 - 1, sz = z + t / 9 - 1;
    sx += sx < 0 ? in.nx : (sx >= in.nx ? -in.nx : 0);
    sy += sy < 0 ? in.ny : (sy >= in.ny ? -in.ny : 0);
    sz += sz < 0 ? in.nz : (sz >= in.nz ? -in.nz : 0);
    return vidx(sx, sy, sz, in);
  } else {  // GATHER2
    return vidx(2 * x + (t & 1), 2 * y + ((t >> 1) & 1), 2 * z + (t >> 2), in);
  }
}

template <int SRC, int DST, int NW, int RF, bool F32, bool RELU>
__global__ void __launch_bounds__(256) k_forward(GemmArgs a, float *part, int kper) {
  // LDS: the weight tiles during the K loop; for BF16 outputs the C tile
  // [64*RF rows][16*NW + 8] afterwards, so that each thread stores whole
  // 16-byte channel groups of one output row
  constexpr int OS = 16 * NW + 8;
  constexpr int kSb = 2 * 16 * NW * kLdsK, kOt = F32 ? 0 : 64 * RF * OS;
  __shared__ __attribute__((aligned(16))) bf16 lds[kSb > kOt ? kSb : kOt];
  auto sb = [&](int buf, int row) { return lds + (buf * 16 * NW + row) * kLdsK; };
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = lane & 15, kb = lane >> 4;
  const int64_t mb = (int64_t)blockIdx.x * (64 * RF) + wv * 16 * RF;
  const int n0 = blockIdx.y * 16 * NW;
  const int ktot = a.taps * a.cin;

  int64_t m[RF];
  bool mv[RF];
  int px[RF], py[RF], pz[RF];
#pragma unroll
  for (int f = 0; f < RF; ++f) {
    m[f] = mb + 16 * f + r;
    mv[f] = m[f] < a.M;
    px[f] = py[f] = pz[f] = 0;
    if constexpr (SRC != LBM_NN_IDENT) {
      const int mm = mv[f] ? (int)m[f] : 0;
      px[f] = mm % a.rows.nx;
      py[f] = (mm / a.rows.nx) % a.rows.ny;
      pz[f] = mm / (a.rows.nx * a.rows.ny);
    }
  }

  // A SCATTER2 block computes all 8 taps of its rows in turn: the taps' fine
  // output voxels interleave, so one block writes whole runs of output rows.
  constexpr int NT = DST == LBM_NN_SCATTER2 ? 8 : 1;
  for (int tfix = 0; tfix < NT; ++tfix) {
    // split K (part != NULL, IDENT dst only): block z takes k in [z kper, (z + 1) kper)
    const int kbeg = DST == LBM_NN_SCATTER2 ? tfix * a.cin : (part ? (int)blockIdx.z * kper : 0);
    const int kend = DST == LBM_NN_SCATTER2 ? kbeg + a.cin : (part ? min(kbeg + kper, ktot) : ktot);

    // weight staging: thread -> (column, 8-wide k group)
    const int scol = tid >> 2, sk = 8 * (tid & 3);
    auto stage = [&](int buf, int k0) {
      if (scol < 16 * NW) {
        const int n = n0 + scol, k = k0 + sk;
        bf16x8 v = {};
        if (n < a.cout && k < kend) v = *reinterpret_cast<const bf16x8 *>(a.w + (int64_t)n * ktot + k);
        *reinterpret_cast<bf16x8 *>(sb(buf, scol) + sk) = v;
      }
    };

    // this lane's k group kk = k0 + 8*kb as (tap t, channel c); each load
    // advances it by one 32-wide K step (zeros past the end)
    int kk = kbeg + 8 * kb;
    int t = kk / a.cin, c = kk - t * a.cin;
    auto load_rows = [&](bf16x8(&dst)[RF]) {
#pragma unroll
      for (int f = 0; f < RF; ++f) {
        dst[f] = bf16x8{};
        if (mv[f] && kk < kend)
          dst[f] = *reinterpret_cast<const bf16x8 *>(a.x + gather_row<SRC>(px[f], py[f], pz[f], m[f], t, a.in_grid) *
                                                               a.ldx + c);
      }
      kk += 32;
      c += 32;
      while (c >= a.cin) {
        c -= a.cin;
        ++t;
      }
    };

    f32x4 acc[RF][NW];
#pragma unroll
    for (int f = 0; f < RF; ++f)
#pragma unroll
      for (int j = 0; j < NW; ++j) acc[f][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    bf16x8 cur[RF];
    load_rows(cur);
    stage(0, kbeg);
    __syncthreads();
    int buf = 0;
    for (int k0 = kbeg; k0 < kend; k0 += 32) {
      if (k0 + 32 < kend) stage(buf ^ 1, k0 + 32);
      bf16x8 nxt[RF];
      load_rows(nxt);
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(sb(buf, 16 * j + r) + 8 * kb);
#pragma unroll
        for (int f = 0; f < RF; ++f) acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur[f], bv, acc[f][j], 0, 0, 0);
      }
#pragma unroll
      for (int f = 0; f < RF; ++f) cur[f] = nxt[f];
      __syncthreads();  // (after the last step: every wavefront's weight reads are done)
      buf ^= 1;
    }

    if (part) {
      // split K: this block's FP32 partial sums, part[z][row][n] (bias, ReLU
      // and gate follow in k_forward_finish)
      float *pz = part + (int64_t)blockIdx.z * a.M * a.cout;
#pragma unroll
      for (int f = 0; f < RF; ++f)
#pragma unroll
        for (int j = 0; j < NW; ++j) {
          const int n = n0 + 16 * j + r;
          if (n >= a.cout) continue;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int64_t mo = mb + 16 * f + 4 * kb + i;
            if (mo < a.M) pz[mo * a.cout + n] = acc[f][j][i];
          }
        }
    } else if constexpr (F32) {
      // FP32 rows (the network's head): one element per lane and row
#pragma unroll
      for (int f = 0; f < RF; ++f) {
#pragma unroll
        for (int j = 0; j < NW; ++j) {
          const int n = n0 + 16 * j + r;
          if (n >= a.cout) continue;
          const float bias = a.bias ? a.bias[n] : 0.f;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int64_t mo = mb + 16 * f + 4 * kb + i;
            if (mo >= a.M) continue;
            float v = acc[f][j][i] + bias;
            if (RELU) v = fmaxf(v, 0.f);
            const int64_t dv = dst_voxel<DST>(mo, tfix, a.rows, a.out_grid);
            if (n < a.gate_ch && !gate_open(a.gate[dv * a.ldg + n])) v = 0.f;
            static_cast<float *>(a.y)[dv * a.ldy + n] = v;
          }
        }
      }
    } else {
      // bias and ReLU, then the tile goes through LDS as [row][channel]
      bf16 *ot = lds;
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        const int n = n0 + 16 * j + r;
        const float bias = (a.bias && n < a.cout) ? a.bias[n] : 0.f;
#pragma unroll
        for (int f = 0; f < RF; ++f)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float v = acc[f][j][i] + bias;
            if (RELU) v = fmaxf(v, 0.f);
            ot[(wv * 16 * RF + 16 * f + 4 * kb + i) * OS + 16 * j + r] = (bf16)v;
          }
      }
      __syncthreads();
      // thread -> (row, 8-channel group); consecutive threads take consecutive
      // groups of one row, then the next row
      for (int e = tid; e < 64 * RF * 2 * NW; e += 256) {
        const int rl = e / (2 * NW), q = e % (2 * NW);
        const int64_t mo = (int64_t)blockIdx.x * (64 * RF) + rl;
        const int n = n0 + 8 * q;
        if (mo >= a.M || n >= a.cout) continue;
        bf16x8 o = *reinterpret_cast<const bf16x8 *>(ot + rl * OS + 8 * q);
        const int64_t dv = dst_voxel<DST>(mo, tfix, a.rows, a.out_grid);
        if (n < a.gate_ch) {  // whole 8-channel groups (gate_ch is a multiple of 8)
          const bf16x8 gv = *reinterpret_cast<const bf16x8 *>(a.gate + dv * a.ldg + n);
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (!gate_open(gv[u])) o[u] = (bf16)0.f;
        }
        *reinterpret_cast<bf16x8 *>(static_cast<bf16 *>(a.y) + dv * a.ldy + n) = o;
      }
      __syncthreads();  // the tile's reads are done before LDS takes weights again
    }
  }
}

// Split-K epilogue: y[row][n] = act(sum over the splits z = 0 .. S-1, in that
// order, of part[z][row][n] + bias[n]), gated like k_forward; BF16 rows, one
// thread per (row, 8-channel group).
template <bool RELU>
__global__ void __launch_bounds__(256) k_forward_finish(GemmArgs a, const float *__restrict__ part, int S) {
  const int groups = a.cout / 8;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= a.M * groups) return;
  const int64_t row = e / groups;
  const int n = 8 * (int)(e % groups);
  float v[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) v[u] = a.bias ? a.bias[n + u] : 0.f;
  float sum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int z = 0; z < S; ++z) {
    const float4 *p = reinterpret_cast<const float4 *>(part + ((int64_t)z * a.M + row) * a.cout + n);
    const float4 lo = p[0], hi = p[1];
    sum[0] += lo.x, sum[1] += lo.y, sum[2] += lo.z, sum[3] += lo.w;
    sum[4] += hi.x, sum[5] += hi.y, sum[6] += hi.z, sum[7] += hi.w;
  }
  bf16x8 o;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    float x = sum[u] + v[u];
    if (RELU) x = fmaxf(x, 0.f);
    o[u] = (bf16)x;
  }
  if (n < a.gate_ch) {
    const bf16x8 gv = *reinterpret_cast<const bf16x8 *>(a.gate + row * a.ldg + n);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (!gate_open(gv[u])) o[u] = (bf16)0.f;
  }
  *reinterpret_cast<bf16x8 *>(static_cast<bf16 *>(a.y) + row * a.ldy + n) = o;
}

// ---- transposed 2x2x2 stride-2 convolution (scatter) forward ---------------
// Every tap reads the same coarse rows, so a block loads its A fragments once
// (all K steps, in registers) and runs its taps in turn: tap t's weight tile
// (16*NW columns x cin) is staged in LDS, double-buffered, with the next tap's
// tile loaded during this tap's MFMAs; the output tile goes through LDS into
// 16-byte stores of the tap's fine voxels.  Block z takes taps
// [z * 8 / gridDim.z, (z + 1) * 8 / gridDim.z) (small grids spread the taps
// over more blocks).  BF16 output; cin <= 32 * KSM.
template <int NW, int RF, bool RELU>
__global__ void __launch_bounds__(256) k_up2(GemmArgs a) {
  constexpr int KSM = 8 / RF;                       // K steps held in registers
  constexpr int OS = 16 * NW + 8;
  constexpr int WPT = (16 * NW * KSM * 4 + 255) / 256;  // weight staging loads per thread
  extern __shared__ __attribute__((aligned(16))) bf16 ulds[];
  const int ks = (a.cin + 31) / 32, wp = 32 * ks + 8;  // K steps; weight tile pitch (bf16)
  bf16 *wbuf = ulds;                                 // [2][16*NW][wp]
  bf16 *ot = ulds + 2 * 16 * NW * wp;                // [64*RF][OS]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = lane & 15, kb = lane >> 4;
  const int64_t rb = (int64_t)blockIdx.x * (64 * RF);  // first row of the block
  const int n0 = blockIdx.y * 16 * NW;
  const int tpb = 8 / gridDim.z, t0 = blockIdx.z * tpb, ktot = 8 * a.cin;

  bf16x8 av[KSM][RF];
#pragma unroll
  for (int st = 0; st < KSM; ++st)
#pragma unroll
    for (int f = 0; f < RF; ++f) {
      const int64_t m = rb + wv * 16 * RF + 16 * f + r;
      const int c = 32 * st + 8 * kb;
      av[st][f] = bf16x8{};
      if (st < ks && m < a.M && c < a.cin) av[st][f] = *reinterpret_cast<const bf16x8 *>(a.x + m * a.ldx + c);
    }

  // weight tile of tap t: entry e = (column, 8-wide k group), zeros past cin and cout
  bf16x8 wreg[WPT];
  const int wgroups = 16 * NW * 4 * ks;
  auto load_w = [&](int t) {
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
      const int e = tid + 256 * u;
      const int col = e / (4 * ks), k = 8 * (e % (4 * ks));
      wreg[u] = bf16x8{};
      if (e < wgroups && n0 + col < a.cout && k < a.cin)
        wreg[u] = *reinterpret_cast<const bf16x8 *>(a.w + (int64_t)(n0 + col) * ktot + t * a.cin + k);
    }
  };
  auto store_w = [&](int buf) {
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
      const int e = tid + 256 * u;
      if (e < wgroups)
        *reinterpret_cast<bf16x8 *>(wbuf + (buf * 16 * NW + e / (4 * ks)) * wp + 8 * (e % (4 * ks))) = wreg[u];
    }
  };

  load_w(t0);
  store_w(0);
  int buf = 0;
  for (int t = t0; t < t0 + tpb; ++t) {
    __syncthreads();  // tap t's weights are staged; the previous tile's reads are done
    if (t + 1 < t0 + tpb) load_w(t + 1);  // in flight during this tap's MFMAs
    f32x4 acc[RF][NW];
#pragma unroll
    for (int f = 0; f < RF; ++f)
#pragma unroll
      for (int j = 0; j < NW; ++j) acc[f][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int st = 0; st < KSM; ++st) {
      if (st >= ks) break;
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(wbuf + (buf * 16 * NW + 16 * j + r) * wp + 32 * st + 8 * kb);
#pragma unroll
        for (int f = 0; f < RF; ++f) acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[st][f], bv, acc[f][j], 0, 0, 0);
      }
    }
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const int n = n0 + 16 * j + r;
      const float bias = (a.bias && n < a.cout) ? a.bias[n] : 0.f;
#pragma unroll
      for (int f = 0; f < RF; ++f)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float v = acc[f][j][i] + bias;
          if (RELU) v = fmaxf(v, 0.f);
          ot[(wv * 16 * RF + 16 * f + 4 * kb + i) * OS + 16 * j + r] = (bf16)v;
        }
    }
    __syncthreads();
    for (int e = tid; e < 64 * RF * 2 * NW; e += 256) {
      const int rl = e / (2 * NW), q = e % (2 * NW);
      const int64_t mo = rb + rl;
      const int n = n0 + 8 * q;
      if (mo >= a.M || n >= a.cout) continue;
      bf16x8 o = *reinterpret_cast<const bf16x8 *>(ot + rl * OS + 8 * q);
      const int64_t dv = dst_voxel<LBM_NN_SCATTER2>(mo, t, a.rows, a.out_grid);
      if (n < a.gate_ch) {
        const bf16x8 gv = *reinterpret_cast<const bf16x8 *>(a.gate + dv * a.ldg + n);
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (!gate_open(gv[u])) o[u] = (bf16)0.f;
      }
      *reinterpret_cast<bf16x8 *>(static_cast<bf16 *>(a.y) + dv * a.ldy + n) = o;
    }
    if (t + 1 < t0 + tpb) store_w(buf ^ 1);
    buf ^= 1;
  }
}

template <int NW, int RF>
hipError_t launch_up2_nw(const GemmArgs &a, bool relu, dim3 grid, size_t lds, hipStream_t s) {
  const void *k = relu ? reinterpret_cast<const void *>(&k_up2<NW, RF, true>)
                       : reinterpret_cast<const void *>(&k_up2<NW, RF, false>);
  hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (relu)
    hipLaunchKernelGGL((k_up2<NW, RF, true>), grid, dim3(256), lds, s, a);
  else
    hipLaunchKernelGGL((k_up2<NW, RF, false>), grid, dim3(256), lds, s, a);
  return hipGetLastError();
}

// ---- CONV3 forward on spatial bricks -----------------------------------------
// A block owns an 8x8x4 brick of output voxels and 16*NW output channels; for
// each chunk of CC input channels it stages the brick's 10x10x6 input halo
// (periodic wrap) in LDS once, and all 27 taps read their A fragments from
// there, so each input row is fetched about 2.3 times per block instead of 27.
// Wavefront w owns the z-plane w of the brick; its fragment f covers rows
// y = 2f, 2f+1 (x = 0..7).  The tap loop is unrolled, so a tap's halo offset
// is an immediate of the LDS read.  With CC = 32 each tap is one K step; CC = 8
// packs four taps into one K step; CC = 24 and 48 run K over (tap, channel)
// flattened.  Weight rows are read straight from global memory at clamped
// addresses: K lanes past the end meet zero A values, and columns past cout
// are never stored.
constexpr int kBrickX = 8, kBrickY = 8, kBrickZ = 4;
constexpr int kHaloX = kBrickX + 2, kHaloY = kBrickY + 2, kHaloZ = kBrickZ + 2;
constexpr int kHalo = kHaloX * kHaloY * kHaloZ;

// Halo layout in LDS (bf16 units): voxel (hx, hy, hz) at hx * CP + (hy + kHaloY hz) * RP.  A fragment's 16 lanes
// read 8 voxels of two y-rows in one LDS cycle (64 banks of 4 bytes): the voxel pitch CP is an odd multiple of 4
// banks, so the 8 voxels of a row take 8 distinct groups of 4 banks, and the row pitch RP is 32 banks modulo 64,
// so the second row takes the other 8 groups.
template <int CC>
struct BrickShape {
  static constexpr int KS = CC == 8 ? 1 : (CC + 31) / 32;  // K steps per tap
  static constexpr int width = CC == 32 ? 32 : CC;          // channels staged per halo voxel (8, 24, 32 or 48)
  static constexpr int CP = CC == 32 ? 40 : (CC == 48 ? 56 : 24);     // voxel pitch: 20, 28 or 12 banks
  static constexpr int RP = CC == 32 ? 448 : (CC == 48 ? 576 : 320);  // row pitch: 224, 288 or 160 banks (32 mod 64)
  static constexpr int ROWS = kHaloY * kHaloZ;
  static_assert(kHaloX * CP <= RP && (RP / 2) % 64 == 32 && (CP / 2) % 8 == 4, "halo layout");
};

template <int CC>
constexpr int tap_off(int t) {
  return (t % 3) * BrickShape<CC>::CP + (((t / 3) % 3) + kHaloY * (t / 9)) * BrickShape<CC>::RP;
}

constexpr int kBrickRing8 = 3;  // K steps of weights loaded ahead in the 8-channel form

// LDS of a brick block in bf16 elements: the halo, or the output tile of 256
// voxels x (16 NW + 8) that reuses it; past 64 KB it is dynamic LDS
template <int NW, int CC>
constexpr int brick_lds() {
  constexpr int halo = BrickShape<CC>::ROWS * BrickShape<CC>::RP, out = kBrickX * kBrickY * kBrickZ * (16 * NW + 8);
  return halo > out ? halo : out;
}
template <int NW, int CC>
constexpr bool brick_dyn() { return brick_lds<NW, CC>() * 2 > 65536; }

template <int NW, int CC, bool RELU>
__global__ void __launch_bounds__(256, (NW <= 2 && CC != 48 ? 4 : 2)) k_conv3_brick(GemmArgs a) {
  using BS = BrickShape<CC>;
  constexpr int CP = BS::CP, RP = BS::RP;
  constexpr int OS = 16 * NW + 8;
  constexpr int kLds = brick_lds<NW, CC>();
  __shared__ __attribute__((aligned(16))) bf16 halo_s[brick_dyn<NW, CC>() ? 8 : kLds];
  extern __shared__ __attribute__((aligned(16))) bf16 halo_dyn[];
  bf16 *const halo = brick_dyn<NW, CC>() ? halo_dyn : halo_s;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = lane & 15, kb = lane >> 4;
  const Grid g = a.rows;  // CONV3: output grid == input grid
  const int bxn = (g.nx + kBrickX - 1) / kBrickX, byn = (g.ny + kBrickY - 1) / kBrickY;
  const int bid = blockIdx.x;
  const int ox = (bid % bxn) * kBrickX, oy = ((bid / bxn) % byn) * kBrickY, oz = (bid / (bxn * byn)) * kBrickZ;
  const int n0 = blockIdx.y * 16 * NW;
  const int ktot = 27 * a.cin;

  // per-lane LDS element offsets of the four fragments' rows at tap (0,0,0)
  int rowbase[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) rowbase[f] = (r & 7) * CP + ((2 * f + (r >> 3)) + kHaloY * wv) * RP;
  // per-lane byte offsets of the weight rows (clamped to a valid output
  // channel) from a uniform base, so each weight load is a scalar base plus
  // a 32-bit lane offset with no per-load address arithmetic
  uint32_t wrow[NW];
#pragma unroll
  for (int j = 0; j < NW; ++j) wrow[j] = (uint32_t)(min(n0 + 16 * j + r, a.cout - 1) * ktot) * 2u;
  auto wload = [&](int k, uint32_t lane_off) {  // k: uniform element offset inside a weight row
    return *reinterpret_cast<const bf16x8 *>(reinterpret_cast<const char *>(a.w + k) + lane_off);
  };

  f32x4 acc[4][NW];
#pragma unroll
  for (int f = 0; f < 4; ++f)
#pragma unroll
    for (int j = 0; j < NW; ++j) acc[f][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  constexpr int G = BS::width / 8;                 // 16-byte groups per halo row that are read
  constexpr int NST = (kHalo * G + 255) / 256;     // staging loads per thread
  // element offsets of the halo's wrapped rows (hy, hz) and columns hx, once
  // per block, so that a staging entry's input row is a sum of two table
  // entries instead of three wraps and a 64-bit index product per entry
  __shared__ int64_t hrow[kHaloY * kHaloZ], hcol[kHaloX];
  if (tid < kHaloY * kHaloZ) {
    const int hy = tid % kHaloY, hz = tid / kHaloY;
    hrow[tid] = ((int64_t)wrap(oy + hy - 1, g.ny) + (int64_t)g.ny * wrap(oz + hz - 1, g.nz)) * g.nx * a.ldx;
  } else if (tid < kHaloY * kHaloZ + kHaloX) {
    const int hx = tid - kHaloY * kHaloZ;
    hcol[hx] = (int64_t)wrap(ox + hx - 1, g.nx) * a.ldx;
  }
  __syncthreads();
  // input row of each of this thread's staging entries (the same for every chunk)
  int64_t srow[NST];
#pragma unroll
  for (int it = 0; it < NST; ++it) {
    const int e = tid + 256 * it;
    const int hv = min(e / G, kHalo - 1);  // entries past the halo load nothing
    srow[it] = hrow[hv / kHaloX] + hcol[hv % kHaloX];
  }
  for (int c0 = 0; c0 < a.cin; c0 += CC) {
    // issue every staging load of the chunk before the first LDS store
    bf16x8 v[NST];
#pragma unroll
    for (int it = 0; it < NST; ++it) {
      const int e = tid + 256 * it;
      const int q = e % G;
      v[it] = bf16x8{};
      if (e < kHalo * G && 8 * q < CC) v[it] = *reinterpret_cast<const bf16x8 *>(a.x + srow[it] + c0 + 8 * q);
    }
    __syncthreads();  // the previous chunk's reads are done
#pragma unroll
    for (int it = 0; it < NST; ++it) {
      const int e = tid + 256 * it;
      if (e < kHalo * G) {
        const int hv = e / G;
        *reinterpret_cast<bf16x8 *>(&halo[(hv % kHaloX) * CP + (hv / kHaloX) * RP + 8 * (e % G)]) = v[it];
      }
    }
    __syncthreads();
    if constexpr (CC == 8) {
      // four taps per K step: lane group kb takes tap 4s + kb (tap 27 is padding)
      bf16x8 ring[kBrickRing8][NW];
      auto load_w = [&](int s0, bf16x8(&dst)[NW]) {
        // lane group kb reads tap s0 + kb (tap 27, the padding, reads tap 26:
        // its A values are zero)
        const uint32_t toff = (uint32_t)((min(s0 + kb, 26) - s0) * a.cin) * 2u;
#pragma unroll
        for (int j = 0; j < NW; ++j) dst[j] = wload(s0 * a.cin + c0, wrow[j] + toff);
      };
      static_for<kBrickRing8>([&](auto P) { load_w(4 * decltype(P)::value, ring[decltype(P)::value]); });
      static_for<7>([&](auto S) {
        constexpr int sidx = decltype(S)::value, s0 = 4 * sidx, slot = sidx % kBrickRing8;
        const int t = s0 + kb;
        const int off = kb == 0 ? tap_off<CC>(s0) : kb == 1 ? tap_off<CC>(s0 + 1)
                      : kb == 2 ? tap_off<CC>(s0 + 2) : tap_off<CC>(s0 + 3 < 27 ? s0 + 3 : 26);
        const bool tv = t < 27;
        bf16x8 bv[NW];
#pragma unroll
        for (int j = 0; j < NW; ++j) bv[j] = ring[slot][j];
        // the weights kBrickRing8 K steps ahead are in flight during these MFMAs
        if constexpr (sidx + kBrickRing8 < 7) load_w(4 * (sidx + kBrickRing8), ring[slot]);
        __builtin_amdgcn_sched_barrier(0);  // keep the load here: the scheduler would sink it next to its use
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          bf16x8 av = *reinterpret_cast<const bf16x8 *>(&halo[rowbase[f] + off]);
          if (!tv) av = bf16x8{};
#pragma unroll
          for (int j = 0; j < NW; ++j)
            acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[j], acc[f][j], 0, 0, 0);
        }
      });
    } else if constexpr (CC == 24 || CC == 48) {
      // 24- and 48-channel chunks: K runs over (tap, channel) flattened, 27 CC
      // = 20.25 or 40.5 K steps of 32 instead of 27 or 54 steps padded to
      // whole 32-channel steps.  Lane group kb of step s takes k = 32 s + 8 kb:
      // channels c .. c + 7 of tap t, with t = t0 + carry and c = c0 + 8 kb - CC
      // carry, where (t0, c0) is lane group 0's (a constant of the step) and
      // carry = (c0 + 8 kb >= CC).  So a lane's LDS offset is a per-step
      // constant plus 8 kb plus a carry term, and its weight offset likewise;
      // the four fragments sit at fixed distances from fragment 0.
      constexpr int NSTEP = (27 * CC + 31) / 32;  // lane groups of the last step past k = 27 CC are zero
      const bool ge1 = kb >= 1, ge2 = kb >= 2, ge3 = kb >= 3;
      auto carry = [&](auto C0) {  // lane group past the tap boundary, for c0 = C0
        constexpr int p = (CC - decltype(C0)::value) / 8;  // first such lane group
        return p == 1 ? ge1 : (p == 2 ? ge2 : (p == 3 ? ge3 : false));
      };
      const int abase = rowbase[0] + 8 * kb;
      const uint32_t wlane = 16u * (uint32_t)kb, wcarry = (uint32_t)(a.cin - CC) * 2u;
      constexpr int R = CC == 48 && NW <= 3 ? 6 : 3;
      bf16x8 ring[R][NW];
      auto load_w = [&](auto U, bf16x8(&dst)[NW]) {
        constexpr int k0 = 32 * decltype(U)::value, t0 = k0 / CC, cc0 = k0 % CC;
        const bool cy = carry(std::integral_constant<int, cc0>{});
        // lanes past the end (last step) read a valid weight; their A is zero
        const bool past = k0 + 8 * kb >= 27 * CC;
        const uint32_t lo = past ? 0u : wlane + (cy ? wcarry : 0u);
#pragma unroll
        for (int j = 0; j < NW; ++j) dst[j] = wload(c0 + t0 * a.cin + cc0, wrow[j] + lo);
      };
      static_for<R>([&](auto P) { load_w(P, ring[decltype(P)::value]); });
      static_for<NSTEP>([&](auto U) {
        constexpr int u = decltype(U)::value, slot = u % R;
        constexpr int k0 = 32 * u, t0 = k0 / CC, cc0 = k0 % CC;
        constexpr int abase_u = tap_off<CC>(t0) + cc0;
        constexpr int acarry = t0 < 26 ? tap_off<CC>(t0 + 1) - tap_off<CC>(t0) - CC : 0;
        const bool cy = carry(std::integral_constant<int, cc0>{});
        const int aoff = abase + (cy ? acarry : 0) + abase_u;
        bf16x8 bv[NW];
#pragma unroll
        for (int j = 0; j < NW; ++j) bv[j] = ring[slot][j];
        if constexpr (u + R < NSTEP) load_w(std::integral_constant<int, u + R>{}, ring[slot]);
        __builtin_amdgcn_sched_barrier(0);  // keep the load here: the scheduler would sink it next to its use
        const bool zero = u == NSTEP - 1 && k0 + 8 * kb >= 27 * CC;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          bf16x8 av = *reinterpret_cast<const bf16x8 *>(&halo[(zero ? abase : aoff) + f * 2 * RP]);
          if (zero) av = bf16x8{};
#pragma unroll
          for (int j = 0; j < NW; ++j)
            acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[j], acc[f][j], 0, 0, 0);
        }
      });
    } else {
      int cb[BS::KS];  // weight channel of this lane's k group, clamped into the tap
#pragma unroll
      for (int st = 0; st < BS::KS; ++st) cb[st] = min(32 * st + 8 * kb, CC - 8);
      // weight fragments of the next R (tap, K step) pairs are loaded ahead
      // into a ring of registers, so their L2 latency overlaps R steps of MFMAs
      constexpr int R = NW <= 2 ? 6 : 3, NSTEP = 27 * BS::KS;
      bf16x8 ring[R][NW];
      auto load_w = [&](int u, bf16x8(&dst)[NW]) {
        const int t = u / BS::KS, st = u % BS::KS;
#pragma unroll
        for (int j = 0; j < NW; ++j) dst[j] = wload(t * a.cin + c0, wrow[j] + (uint32_t)cb[st] * 2u);
      };
      static_for<R>([&](auto P) { load_w(decltype(P)::value, ring[decltype(P)::value]); });
      static_for<NSTEP>([&](auto U) {
        constexpr int u = decltype(U)::value, t = u / BS::KS, st = u % BS::KS, slot = u % R;
        constexpr int off = tap_off<CC>(t);
        bf16x8 bv[NW];
#pragma unroll
        for (int j = 0; j < NW; ++j) bv[j] = ring[slot][j];
        if constexpr (u + R < NSTEP) load_w(u + R, ring[slot]);
        __builtin_amdgcn_sched_barrier(0);  // keep the load here: the scheduler would sink it next to its use
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const bf16x8 av = *reinterpret_cast<const bf16x8 *>(&halo[rowbase[f] + off + 32 * st + 8 * kb]);
#pragma unroll
          for (int j = 0; j < NW; ++j)
            acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[j], acc[f][j], 0, 0, 0);
        }
      });
    }
  }

  // epilogue: bias and ReLU, then the tile goes through LDS as [voxel][channel]
  // so that each thread writes whole 16-byte channel groups of one voxel
  __syncthreads();  // every wavefront's last halo reads are done
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    const int nl = 16 * j + r, n = n0 + nl;
    const float bias = (a.bias && n < a.cout) ? a.bias[n] : 0.f;
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = 4 * kb + i;  // row of the fragment: x = q & 7, y = 2f + (q >> 3), z = wv
        float v = acc[f][j][i] + bias;
        if (RELU) v = fmaxf(v, 0.f);
        halo[((q & 7) + kBrickX * (2 * f + (q >> 3) + kBrickY * wv)) * OS + nl] = (bf16)v;
      }
  }
  __syncthreads();
  const int x = ox + (tid & 7), y = oy + ((tid >> 3) & 7), z = oz + (tid >> 6);
  if (x < g.nx && y < g.ny && z < g.nz) {
    const int64_t v = vidx(x, y, z, g);
    bf16 *dst = static_cast<bf16 *>(a.y) + v * a.ldy + n0;
#pragma unroll
    for (int c = 0; c < 2 * NW; ++c)
      if (n0 + 8 * c < a.cout) {
        bf16x8 o = *reinterpret_cast<const bf16x8 *>(&halo[tid * OS + 8 * c]);
        if (n0 + 8 * c < a.gate_ch) {  // whole 8-channel groups (gate_ch is a multiple of 8)
          const bf16x8 gv = *reinterpret_cast<const bf16x8 *>(a.gate + v * a.ldg + n0 + 8 * c);
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (!gate_open(gv[e])) o[e] = (bf16)0.f;
        }
        *reinterpret_cast<bf16x8 *>(dst + 8 * c) = o;
      }
  }
}

// The transposing LDS load of gfx950 (ds_read_b64_tr_b16): in each group of
// 16 lanes, lane L supplies the address of 4 consecutive bf16, here channels
// 4 (L % 4) .. 4 (L % 4) + 3 of row L / 4 of a [row][channel] tile, and lane j
// receives element r of it from lane 4 r + j / 4, element j % 4: channel j of
// rows 0-3.  Two such loads give a lane the 8 K values of one MFMA operand row.
typedef short v4s16 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v4s16 lds_v4s16;

// The 8 K values of one MFMA operand row from two transposing LDS loads: p0
// and p1 are this lane's addresses for voxels 0-3 and 4-7 of its K group.
__device__ __forceinline__ bf16x8 tr_load8(const bf16 *p0, const bf16 *p1) {
  const v4s16 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s16 *)(p0));
  const v4s16 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s16 *)(p1));
  typedef short v8s16 __attribute__((ext_vector_type(8)));
  const v8s16 v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  return __builtin_bit_cast(bf16x8, v);
}

// ---- weight gradient: voxels are the reduction ------------------------------
// Block: tap t, 16*CF input channels, 16*NF output channels, a voxel chunk.
// Each wavefront stages 32 voxels of x and dy in LDS as they are stored
// ([voxel][channel], 16-byte writes) and reads its MFMA operands with the
// transposing LDS load (tr_load8: channel r of the 8 voxels of K group kb); it
// runs CF x NF MFMAs per 32 voxels, and the four wavefronts' sums meet in LDS
// at the end.
constexpr int kWgradPad = 8;  // bf16 of padding per LDS row

// 32-bit row -> voxel maps (grids are checked to hold fewer than 2^31 rows)
template <int SRC>
__device__ __forceinline__ int64_t src_voxel32(int m, int t, const Grid &rows, const Grid &in) {
  if constexpr (SRC == LBM_NN_IDENT) {
    return m;
  } else {
    const int x = m % rows.nx, y = (m / rows.nx) % rows.ny, z = m / (rows.nx * rows.ny);
    return gather_row<SRC>(x, y, z, m, t, in);
  }
}

template <int DST>
__device__ __forceinline__ int64_t dst_voxel32(int m, int t, const Grid &rows, const Grid &out) {
  if constexpr (DST == LBM_NN_IDENT) {
    return m;
  } else {
    const int x = m % rows.nx, y = (m / rows.nx) % rows.ny, z = m / (rows.nx * rows.ny);
    return vidx(2 * x + (t & 1), 2 * y + ((t >> 1) & 1), 2 * z + (t >> 2), out);
  }
}

// LDS written by this wavefront's lanes is visible to its other lanes
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Each wavefront stages its own 32 voxels per iteration (LDS tiles private to
// the wave, so only wave-level synchronisation), and the next iteration's
// rows are loaded into registers while the current MFMAs run.
template <int SRC, int DST, int CF, int NF>
__global__ void __launch_bounds__(256) k_wgrad(GemmArgs a, float *dw, int64_t chunk, int cblocks, float *ws,
                                               float *db) {
  __shared__ __attribute__((aligned(16))) bf16 sx[4][32][16 * CF + kWgradPad];
  __shared__ __attribute__((aligned(16))) bf16 sy[4][32][16 * NF + kWgradPad];
  __shared__ float red[4][16 * CF][16 * NF + 1];
  __shared__ float bred[4][16 * NF];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = lane & 15, kb = lane >> 4;
  // transposing loads: this lane supplies voxel 8 kb + tv (and + 4), channels 4 tq ..
  const int tv = r >> 2, tq = r & 3;
  const int t = blockIdx.y % a.taps, cb = blockIdx.y / a.taps, nb = blockIdx.z;
  // bias gradient (with db): the blocks of the first input-channel tile sum
  // their dy rows, each output row once (every tap of a scatter writes its own
  // fine voxels; the other layers' taps share one output row)
  const bool bias = db && cb == 0 && (DST == LBM_NN_SCATTER2 || t == 0);
  float bsum[NF];
#pragma unroll
  for (int j = 0; j < NF; ++j) bsum[j] = 0.f;
  const int cbase = cb * 16 * CF, nbase = nb * 16 * NF;
  const int64_t v0 = (int64_t)blockIdx.x * chunk;
  int64_t v1 = v0 + chunk;
  if (v1 > a.M) v1 = a.M;
  const int vl = lane & 31, g0 = lane >> 5;  // staging: voxel and first 8-channel group of this lane

  auto load = [&](int64_t vb, bf16x8(&xv)[CF], bf16x8(&yv)[NF]) {
    const int64_t m = vb + 32 * wv + vl;
    const bool mv = m < v1;
    const int mm = mv ? (int)m : 0;
    const bf16 *xr = a.x + src_voxel32<SRC>(mm, t, a.rows, a.in_grid) * a.ldx;
    const bf16 *yr = static_cast<const bf16 *>(a.y) + dst_voxel32<DST>(mm, t, a.rows, a.out_grid) * a.ldy;
#pragma unroll
    for (int g = 0; g < CF; ++g) {
      const int c = cbase + 8 * (g0 + 2 * g);
      xv[g] = bf16x8{};
      if (mv && c < a.cin) xv[g] = *reinterpret_cast<const bf16x8 *>(xr + c);
    }
#pragma unroll
    for (int g = 0; g < NF; ++g) {
      const int n = nbase + 8 * (g0 + 2 * g);
      yv[g] = bf16x8{};
      if (mv && n < a.cout) yv[g] = *reinterpret_cast<const bf16x8 *>(yr + n);
    }
  };

  f32x4 acc[CF][NF];
#pragma unroll
  for (int i = 0; i < CF; ++i)
#pragma unroll
    for (int j = 0; j < NF; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  bf16x8 xv[CF], yv[NF];
  if (v0 < v1) load(v0, xv, yv);
  for (int64_t vb = v0; vb < v1; vb += 128) {
#pragma unroll
    for (int g = 0; g < CF; ++g) *reinterpret_cast<bf16x8 *>(&sx[wv][vl][8 * (g0 + 2 * g)]) = xv[g];
#pragma unroll
    for (int g = 0; g < NF; ++g) *reinterpret_cast<bf16x8 *>(&sy[wv][vl][8 * (g0 + 2 * g)]) = yv[g];
    wave_lds_sync();
    if (vb + 128 < v1) load(vb + 128, xv, yv);  // in flight during the MFMAs
    bf16x8 bv[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j)
      bv[j] = tr_load8(&sy[wv][8 * kb + tv][16 * j + 4 * tq], &sy[wv][8 * kb + 4 + tv][16 * j + 4 * tq]);
    if (bias)  // lane (r, kb) holds channel 16 j + r of the 8 voxels of K group kb
#pragma unroll
      for (int j = 0; j < NF; ++j)
#pragma unroll
        for (int q = 0; q < 8; ++q) bsum[j] += (float)bv[j][q];
#pragma unroll
    for (int i = 0; i < CF; ++i) {
      const bf16x8 av = tr_load8(&sx[wv][8 * kb + tv][16 * i + 4 * tq], &sx[wv][8 * kb + 4 + tv][16 * i + 4 * tq]);
#pragma unroll
      for (int j = 0; j < NF; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[j], acc[i][j], 0, 0, 0);
    }
    wave_lds_sync();  // this wave's reads are done before its next staging
  }
  // lane holds C[c = 16i + 4kb + q][n = 16j + r]
#pragma unroll
  for (int i = 0; i < CF; ++i)
#pragma unroll
    for (int j = 0; j < NF; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) red[wv][16 * i + 4 * kb + q][16 * j + r] = acc[i][j][q];
  if (bias) {  // (uniform per block) the K groups, then the wavefronts, meet; one atomic add per channel
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      float v = bsum[j];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (kb == 0) bred[wv][16 * j + r] = v;
    }
  }
  __syncthreads();
  if (bias && threadIdx.x < 16 * NF && nbase + (int)threadIdx.x < a.cout)
    atomicAdd(db + nbase + threadIdx.x, (bred[0][threadIdx.x] + bred[1][threadIdx.x]) +
                                            (bred[2][threadIdx.x] + bred[3][threadIdx.x]));
  // the block's sums: with a workspace into its own slot [16*CF][16*NF] (slots
  // ordered [tile = (nb, cb, t)][chunk]; k_wgrad_sum adds the chunks in a fixed
  // order), else one FP32 atomic add per weight
  const int ktot = a.taps * a.cin;
  float *slot = ws ? ws + (((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * (256 * CF * NF)
                   : nullptr;
  for (int e = threadIdx.x; e < 256 * CF * NF; e += 256) {
    const int cl = e / (16 * NF), nl = e % (16 * NF);
    const float s = red[0][cl][nl] + red[1][cl][nl] + red[2][cl][nl] + red[3][cl][nl];
    if (slot) {
      slot[e] = s;
      continue;
    }
    const int c = cbase + cl, n = nbase + nl;
    if (c >= a.cin || n >= a.cout) continue;
    atomicAdd(dw + (int64_t)n * ktot + (int64_t)t * a.cin + c, s);
  }
}

// ---- weight gradient of the transposed 2x2x2 stride-2 convolution ----------
// dW[n][t][c] += sum over coarse rows m of x[m][c] * dy[fine(m, t)][n].  A
// block of 8 wavefronts takes a chunk of coarse rows and one channel tile;
// wavefront w computes tap w.  Per 64 rows the block stages the x rows once in
// LDS (shared by the 8 taps) and each wavefront its own tap's dy rows, both as
// stored, and reads the MFMA operands with the transposing load.  So x is read
// once instead of once per tap.  Partial sums as in k_wgrad_brick (slot
// [8][16*CF][16*NF] per block) or FP32 atomics; with db the bias gradient too.
template <int CF, int NF>
__global__ void __launch_bounds__(512) k_wgrad_up2(GemmArgs a, float *dw, int chunk, int cblocks, float *ws,
                                                   float *db) {
  constexpr int V = 64, PX = 16 * CF + 8, PY = 16 * NF + 8;
  constexpr int NX = (V * 2 * CF + 511) / 512, NY = 2 * NF;  // x loads per thread (block), dy loads per lane (wave)
  __shared__ __attribute__((aligned(16))) bf16 sx[V * PX];
  __shared__ __attribute__((aligned(16))) bf16 sy[8][V * PY];
  __shared__ float bred[8][16 * NF];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // the tap
  const int r = lane & 15, kb = lane >> 4, tv = r >> 2, tq = r & 3;
  const int cbase = (blockIdx.y % cblocks) * 16 * CF, nbase = (blockIdx.y / cblocks) * 16 * NF;
  const int v0 = blockIdx.x * chunk, v1 = min(v0 + chunk, (int)a.M);
  const bool bias = db && blockIdx.y % cblocks == 0;
  const bf16 *__restrict__ dy = static_cast<const bf16 *>(a.y);

  f32x4 acc[CF][NF];
#pragma unroll
  for (int i = 0; i < CF; ++i)
#pragma unroll
    for (int j = 0; j < NF; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum[NF];
#pragma unroll
  for (int j = 0; j < NF; ++j) bsum[j] = 0.f;

  bf16x8 xv[NX], yv[NY];
  // rows vb .. vb + 63: x entry e = (row e / 2CF, 8-channel group e % 2CF); dy
  // of tap w: lane l takes row l, groups 0 .. 2NF-1 (zeros past the ends)
  auto load = [&](int vb) {
#pragma unroll
    for (int u = 0; u < NX; ++u) {
      const int e = tid + 512 * u, m = vb + e / (2 * CF), c = cbase + 8 * (e % (2 * CF));
      xv[u] = bf16x8{};
      if (e < V * 2 * CF && m < v1 && c < a.cin) xv[u] = *reinterpret_cast<const bf16x8 *>(a.x + (int64_t)m * a.ldx + c);
    }
    const int m = vb + lane;
    const int64_t fy = m < v1 ? dst_voxel32<LBM_NN_SCATTER2>(m, w, a.rows, a.out_grid) * a.ldy : 0;
#pragma unroll
    for (int g = 0; g < NY; ++g) {
      const int n = nbase + 8 * g;
      yv[g] = bf16x8{};
      if (m < v1 && n < a.cout) yv[g] = *reinterpret_cast<const bf16x8 *>(dy + fy + n);
    }
  };

  if (v0 < v1) load(v0);
  for (int vb = v0; vb < v1; vb += V) {
    __syncthreads();  // the previous rows' LDS reads are done
#pragma unroll
    for (int u = 0; u < NX; ++u) {
      const int e = tid + 512 * u;
      if (e < V * 2 * CF) *reinterpret_cast<bf16x8 *>(&sx[(e / (2 * CF)) * PX + 8 * (e % (2 * CF))]) = xv[u];
    }
#pragma unroll
    for (int g = 0; g < NY; ++g) *reinterpret_cast<bf16x8 *>(&sy[w][lane * PY + 8 * g]) = yv[g];
    __syncthreads();
    if (vb + V < v1) load(vb + V);  // in flight during the MFMAs
#pragma unroll
    for (int ks = 0; ks < V / 32; ++ks) {
      const int row = 32 * ks + 8 * kb + tv;  // this lane's voxel (and + 4) for the transposing loads
      bf16x8 bv[NF];
#pragma unroll
      for (int j = 0; j < NF; ++j)
        bv[j] = tr_load8(&sy[w][row * PY + 16 * j + 4 * tq], &sy[w][(row + 4) * PY + 16 * j + 4 * tq]);
      if (bias)
#pragma unroll
        for (int j = 0; j < NF; ++j)
#pragma unroll
          for (int q = 0; q < 8; ++q) bsum[j] += (float)bv[j][q];
#pragma unroll
      for (int i = 0; i < CF; ++i) {
        const bf16x8 av = tr_load8(&sx[row * PX + 16 * i + 4 * tq], &sx[(row + 4) * PX + 16 * i + 4 * tq]);
#pragma unroll
        for (int j = 0; j < NF; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[j], acc[i][j], 0, 0, 0);
      }
    }
  }
  // lane holds C[c = 16i + 4kb + q][n = 16j + r] of tap w
  float *slot = ws ? ws + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * (8 * 256 * CF * NF) : nullptr;
#pragma unroll
  for (int i = 0; i < CF; ++i)
#pragma unroll
    for (int j = 0; j < NF; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int cl = 16 * i + 4 * kb + q, nl = 16 * j + r;
        if (slot) {
          slot[(w * 16 * CF + cl) * 16 * NF + nl] = acc[i][j][q];
        } else {
          const int c = cbase + cl, n = nbase + nl;
          if (c < a.cin && n < a.cout) atomicAdd(dw + ((int64_t)n * 8 + w) * a.cin + c, acc[i][j][q]);
        }
      }
  if (bias) {  // (uniform per block) K groups, then taps, meet; one atomic add per channel
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      float v = bsum[j];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (kb == 0) bred[w][16 * j + r] = v;
    }
    __syncthreads();
    if (tid < 16 * NF && nbase + tid < a.cout) {
      float t = 0.f;
#pragma unroll
      for (int k = 0; k < 8; ++k) t += bred[k][tid];
      atomicAdd(db + nbase + tid, t);
    }
  }
}

// ---- weight gradient of a 3x3x3 convolution on spatial bricks ---------------
// dW[n][t][c] += sum over output voxels v of x(v + o_t)[c] * dy(v)[n].  The
// voxel-chunk kernel above gathers x and dy once per tap, so a large grid is
// read 27 times; here a block owns a channel tile (16*CF input and 16*NF
// output channels) and a run of 8x4x4-voxel bricks, and for each brick stages
// the 10x6x6 input halo and the brick's dy in LDS once for all 27 taps.
// The reduction (K) runs over voxels while the rows are channels-last, so an
// MFMA operand needs each lane's 8 K values from 8 different voxels.  The
// tiles are staged as they are stored ([voxel][channel], one 16-byte LDS
// write per 8 channels) and read with gfx950's transposing LDS load
// (ds_read_b64_tr_b16): in each group of 16 lanes, lane L supplies the address
// of 4 channels (4 (L % 4) ..) of voxel L / 4, and lane j receives channel j
// of those 4 voxels.  Two such loads give a lane channel j of the 8 voxels of
// one x-row: the A (x) or B (dy) fragment of one K group.  A tap's shift is
// only an address offset into the halo.
// K step k is the brick's z-plane k and lane group g its y-row g.
// Wavefront w accumulates the taps w, w + 4, ... (7 or 6 of them) for the
// whole channel tile in registers; the next brick's global rows are loaded
// while the current brick's MFMAs run.
constexpr int kWbX = 8, kWbY = 4, kWbZ = 4;             // brick (output voxels)
constexpr int kWhX = kWbX + 2, kWhY = kWbY + 2, kWhZ = kWbZ + 2;  // halo extent
constexpr int kWHalo = kWhX * kWhY * kWhZ;              // 360 halo voxels

// W wavefronts per block (4, or 8 for the wider channel tiles, so that the
// accumulators of a wavefront's taps leave room for two wavefronts per SIMD);
// wavefront w takes the taps w, w + W, ... (TAPS or TAPS - 1 of them).
template <int CF, int NF>
struct WBrick {
  static constexpr int W = CF * NF <= 4 ? 4 : 8, T = 64 * W;       // wavefronts, threads
  static constexpr int TAPS = (27 + W - 1) / W, FULL = 27 - (TAPS - 1) * W;  // FULL wavefronts take TAPS taps
  static constexpr int GX = 2 * CF, GY = 2 * NF;                    // 8-channel groups per voxel
  static constexpr int NSX = (kWHalo * GX + T - 1) / T;             // staging loads per thread
  static constexpr int NSY = (kWbX * kWbY * kWbZ * GY + T - 1) / T;
  static constexpr int PX = 16 * CF + 8, PY = 16 * NF + 8;          // voxel pitches (bf16), 16-byte rows
  static constexpr int LDS = (kWHalo * PX + kWbX * kWbY * kWbZ * PY) * 2;  // bytes
};


template <int CF, int NF>
__global__ void __launch_bounds__((CF * NF <= 4 ? 256 : 512), 2) k_wgrad_brick(GemmArgs a, float *dw, int bricks_per_block,
                                                                       int cblocks, float *ws, float *db) {
  using WB = WBrick<CF, NF>;
  extern __shared__ __attribute__((aligned(16))) bf16 wlds[];
  bf16 *xs = wlds;                          // [kWHalo][PX]: halo voxel (hx + 10 (hy + 6 hz))
  bf16 *ys = wlds + kWHalo * WB::PX;        // [128][PY]: brick voxel (x + 8 (y + 4 z))
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: the tap branches below stay scalar
  const int r = lane & 15, g = lane >> 4;
  // transposing loads: this lane supplies voxel tv (and tv + 4) of its x-row, channels 4 tq ..
  const int tv = (lane & 15) >> 2, tq = lane & 3;
  const Grid gr = a.rows;  // CONV3: input grid == output grid
  const int cbase = (blockIdx.y % cblocks) * 16 * CF, nbase = (blockIdx.y / cblocks) * 16 * NF;
  const int bxn = (gr.nx + kWbX - 1) / kWbX, byn = (gr.ny + kWbY - 1) / kWbY, bzn = (gr.nz + kWbZ - 1) / kWbZ;
  const int nbricks = bxn * byn * bzn;
  const int b0 = blockIdx.x * bricks_per_block;
  const int b1 = min(b0 + bricks_per_block, nbricks);
  const bf16 *__restrict__ dy = static_cast<const bf16 *>(a.y);

  f32x4 acc[WB::TAPS][CF][NF];
#pragma unroll
  for (int m = 0; m < WB::TAPS; ++m)
#pragma unroll
    for (int i = 0; i < CF; ++i)
#pragma unroll
      for (int j = 0; j < NF; ++j) acc[m][i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  bf16x8 vx[WB::NSX], vy[WB::NSY];
  // global rows of brick b into registers (zeros past the channel counts and
  // for output voxels outside the grid); consecutive threads take consecutive
  // 8-channel groups of one voxel
  auto load = [&](int b) {
    const int ox = (b % bxn) * kWbX, oy = ((b / bxn) % byn) * kWbY, oz = (b / (bxn * byn)) * kWbZ;
#pragma unroll
    for (int it = 0; it < WB::NSX; ++it) {
      const int e = tid + WB::T * it;
      vx[it] = bf16x8{};
      if (e < kWHalo * WB::GX) {
        const int hv = e / WB::GX, q = e % WB::GX;
        const int hx = hv % kWhX, hy = (hv / kWhX) % kWhY, hz = hv / (kWhX * kWhY);
        const int c = cbase + 8 * q;
        if (c < a.cin)
          vx[it] = *reinterpret_cast<const bf16x8 *>(
              a.x + vidx(wrap(ox + hx - 1, gr.nx), wrap(oy + hy - 1, gr.ny), wrap(oz + hz - 1, gr.nz), gr) * a.ldx + c);
      }
    }
#pragma unroll
    for (int it = 0; it < WB::NSY; ++it) {
      const int e = tid + WB::T * it;
      vy[it] = bf16x8{};
      if (e < kWbX * kWbY * kWbZ * WB::GY) {
        const int v = e / WB::GY, q = e % WB::GY;
        const int x = ox + v % kWbX, y = oy + (v / kWbX) % kWbY, z = oz + v / (kWbX * kWbY);
        const int n = nbase + 8 * q;
        if (x < gr.nx && y < gr.ny && z < gr.nz && n < a.cout)
          vy[it] = *reinterpret_cast<const bf16x8 *>(dy + vidx(x, y, z, gr) * a.ldy + n);
      }
    }
  };
  // registers -> LDS as stored: [voxel][channel], one 16-byte write per group
  auto stage = [&]() {
#pragma unroll
    for (int it = 0; it < WB::NSX; ++it) {
      const int e = tid + WB::T * it;
      if (e < kWHalo * WB::GX)
        *reinterpret_cast<bf16x8 *>(xs + (e / WB::GX) * WB::PX + 8 * (e % WB::GX)) = vx[it];
    }
#pragma unroll
    for (int it = 0; it < WB::NSY; ++it) {
      const int e = tid + WB::T * it;
      if (e < kWbX * kWbY * kWbZ * WB::GY)
        *reinterpret_cast<bf16x8 *>(ys + (e / WB::GY) * WB::PY + 8 * (e % WB::GY)) = vy[it];
    }
  };

  // bias gradient (with db, on the blocks of the first input-channel tile):
  // thread -> column bc of the output tile and every BL-th voxel of each brick
  constexpr int BC = 16 * NF, BL = WB::T / BC;
  const bool bias = db && blockIdx.y % cblocks == 0;
  const int bc = tid % BC, bl = tid / BC;
  float bsum = 0.f;

  if (b0 < b1) load(b0);
  for (int b = b0; b < b1; ++b) {
    __syncthreads();  // the previous brick's LDS reads are done
    stage();
    __syncthreads();
    if (b + 1 < b1) load(b + 1);  // in flight during the MFMAs
    if (bias && bl < BL)
      for (int v = bl; v < kWbX * kWbY * kWbZ; v += BL) bsum += (float)ys[v * WB::PY + bc];
#pragma unroll
    for (int k = 0; k < kWbZ; ++k) {
      bf16x8 bv[NF];
      const bf16 *yrow = ys + (tv + kWbX * (g + kWbY * k)) * WB::PY + 4 * tq;
#pragma unroll
      for (int j = 0; j < NF; ++j) bv[j] = tr_load8(yrow + 16 * j, yrow + 4 * WB::PY + 16 * j);
      auto tap = [&](int m) {
        const int t = wv + WB::W * m;
        const int tx = t % 3, ty = (t / 3) % 3, tz = t / 9;
        const bf16 *xrow = xs + ((tv + tx) + kWhX * ((g + ty) + kWhY * (k + tz))) * WB::PX + 4 * tq;
#pragma unroll
        for (int i = 0; i < CF; ++i) {
          const bf16x8 av = tr_load8(xrow + 16 * i, xrow + 4 * WB::PX + 16 * i);
#pragma unroll
          for (int j = 0; j < NF; ++j)
            acc[m][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[j], acc[m][i][j], 0, 0, 0);
        }
      };
      // taps wv + W m < 27 for m < TAPS - 1 on every wavefront; the last one
      // only on wavefronts below FULL (one uniform branch)
#pragma unroll
      for (int m = 0; m < WB::TAPS - 1; ++m) tap(m);
      if (wv < WB::FULL) tap(WB::TAPS - 1);
    }
  }
  if (bias) {  // (uniform per block) the voxel lanes meet in LDS; one atomic add per column
    float *red = reinterpret_cast<float *>(wlds);
    __syncthreads();  // the last brick's LDS reads are done
    red[tid] = bl < BL ? bsum : 0.f;
    __syncthreads();
    if (tid < BC && nbase + tid < a.cout) {
      float t = 0.f;
      for (int l = 0; l < BL; ++l) t += red[l * BC + tid];
      atomicAdd(db + nbase + tid, t);
    }
  }
  // lane holds C[c = 16i + 4g + q][n = 16j + r] of tap t.  With a workspace,
  // the block's partial sums go to its own slot [27][16*CF][16*NF] there and
  // k_wgrad_sum adds the blocks in a fixed order; without one, each weight
  // takes one FP32 atomic add per block.
  const int ktot = 27 * a.cin;
  float *slot = ws ? ws + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * (27 * 256 * CF * NF) : nullptr;
#pragma unroll
  for (int m = 0; m < WB::TAPS; ++m) {
    const int t = wv + WB::W * m;
    if (t >= 27) continue;
#pragma unroll
    for (int i = 0; i < CF; ++i)
#pragma unroll
      for (int j = 0; j < NF; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int cl = 16 * i + 4 * g + q, nl = 16 * j + r;
          if (slot) {
            slot[(t * 16 * CF + cl) * 16 * NF + nl] = acc[m][i][j][q];
          } else {
            const int c = cbase + cl, n = nbase + nl;
            if (c < a.cin && n < a.cout) atomicAdd(dw + (int64_t)n * ktot + (int64_t)t * a.cin + c, acc[m][i][j][q]);
          }
        }
  }
}

// dw += the sum over the blocks of one tile of their partial slots, in two
// passes with a fixed order (run to run identical).  A slot holds slot_taps
// taps x [16*cf][16*nf]: all 27 taps for the brick kernel (tiles = channel
// tiles cb + cblocks * nb), one tap for k_wgrad (tiles = t + taps * (cb +
// cblocks * nb)).  Pass 1: thread (e, part) sums the slots of blocks
// part*per .. part*per + per - 1 with eight independent partial sums (eight
// loads in flight) and writes the total into the first of those slots, which
// only it reads.  Pass 2: thread e adds the parts' totals in order into dw.
// Pass 0 (at most per blocks): pass 1's sum of all blocks, added into dw.
__global__ void __launch_bounds__(256) k_wgrad_sum(float *__restrict__ ws, int blocks, int per, int cf, int nf,
                                                   int cblocks, int slot_taps, int taps, int cin, int cout, float *dw,
                                                   int pass) {
  const int E = slot_taps * 256 * cf * nf;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= E) return;
  const int parts = (blocks + per - 1) / per;
  float sum = 0.f;
  if (pass != 2) {
    const int tile = pass == 1 ? blockIdx.y / parts : blockIdx.y, part = pass == 1 ? blockIdx.y % parts : 0;
    float *p = ws + ((int64_t)tile * blocks + (int64_t)part * per) * E + e;
    const int n = min(per, blocks - part * per);
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int b = 0;
    for (; b + 8 <= n; b += 8)
#pragma unroll
      for (int k = 0; k < 8; ++k) acc[k] += p[(int64_t)(b + k) * E];
    for (; b < n; ++b) acc[0] += p[(int64_t)b * E];
    sum = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    if (pass == 1) {
      p[0] = sum;
      return;
    }
  }
  const int tile = blockIdx.y;
  const int nl = e % (16 * nf), cl = (e / (16 * nf)) % (16 * cf), ts = e / (256 * cf * nf);
  const int ct = slot_taps == taps ? tile : tile / taps;  // channel tile cb + cblocks * nb
  const int t = slot_taps == taps ? ts : tile % taps;
  const int c = (ct % cblocks) * 16 * cf + cl, n = (ct / cblocks) * 16 * nf + nl;
  if (c >= cin || n >= cout) return;
  if (pass == 2) {
    const float *p = ws + (int64_t)tile * blocks * E + e;
    for (int q = 0; q < parts; ++q) sum += p[(int64_t)q * per * E];
  }
  dw[((int64_t)n * taps + t) * cin + c] += sum;
}

// k_wgrad_sum over `tiles` tiles of `blocks` slots each: one pass for at most
// 32 blocks, else two
hipError_t launch_wgrad_sum(float *ws, int64_t blocks, int64_t tiles, int cf, int nf, int cblocks, int slot_taps,
                            int taps, int cin, int cout, float *dw, hipStream_t s) {
  const int E = slot_taps * 256 * cf * nf, per = 32, parts = (int)((blocks + per - 1) / per);
  if (parts == 1) {
    hipLaunchKernelGGL(k_wgrad_sum, dim3((unsigned)((E + 255) / 256), (unsigned)tiles), dim3(256), 0, s, ws,
                       (int)blocks, per, cf, nf, cblocks, slot_taps, taps, cin, cout, dw, 0);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_wgrad_sum, dim3((unsigned)((E + 255) / 256), (unsigned)(tiles * parts)), dim3(256), 0, s, ws,
                     (int)blocks, per, cf, nf, cblocks, slot_taps, taps, cin, cout, dw, 1);
  hipLaunchKernelGGL(k_wgrad_sum, dim3((unsigned)((E + 255) / 256), (unsigned)tiles), dim3(256), 0, s, ws,
                     (int)blocks, per, cf, nf, cblocks, slot_taps, taps, cin, cout, dw, 2);
  return hipGetLastError();
}

// Several layers' backward-data weights in one launch: jobs in the kernel
// argument, block b works on the job whose block range [first, first + blocks)
// holds it.
struct WtJobs {
  lbm_nn_wt_job job[LBM_NN_WT_JOBS_MAX];
  int first[LBM_NN_WT_JOBS_MAX + 1];
  int count;
};

__global__ void __launch_bounds__(256) k_backward_weights_batch(WtJobs J) {
  int j = 0;
  while (j + 1 < J.count && (int)blockIdx.x >= J.first[j + 1]) ++j;
  const lbm_nn_wt_job &b = J.job[j];
  const int taps = b.taps, cin = b.cin, cout = b.cout;
  const int64_t total = (int64_t)taps * cin * cout;
  const int64_t e = (int64_t)(blockIdx.x - J.first[j]) * 256 + threadIdx.x;
  if (e >= total) return;
  // e indexes wt[c][t*cout + n]
  const int c = (int)(e / ((int64_t)taps * cout));
  const int rem = (int)(e % ((int64_t)taps * cout));
  const int t = rem / cout, n = rem % cout;
  const int ts = b.mode == LBM_NN_CONV3 ? (taps - 1 - t) : t;
  static_cast<bf16 *>(b.wt)[e] = static_cast<const bf16 *>(b.w)[(int64_t)n * taps * cin + (int64_t)ts * cin + c];
}

__global__ void k_backward_weights(int mode, int taps, int cin, int cout, const bf16 *w, bf16 *wt) {
  const int64_t total = (int64_t)taps * cin * cout;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    // e indexes wt[c][t*cout + n]
    const int c = (int)(e / ((int64_t)taps * cout));
    const int rem = (int)(e % ((int64_t)taps * cout));
    const int t = rem / cout, n = rem % cout;
    const int ts = mode == LBM_NN_CONV3 ? (taps - 1 - t) : t;
    wt[e] = w[(int64_t)n * taps * cin + (int64_t)ts * cin + c];
  }
}

__global__ void k_maxpool(Grid g, int channels, const bf16 *x, int ldx, bf16 *y, int ldy, uint8_t *arg) {
  const int64_t total = (int64_t)g.nx * g.ny * g.nz * channels;
  const Grid f{2 * g.nx, 2 * g.ny, 2 * g.nz};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % channels);
    const int64_t v = e / channels;
    const int xx = (int)(v % g.nx), yy = (int)((v / g.nx) % g.ny), zz = (int)(v / ((int64_t)g.nx * g.ny));
    float best = -INFINITY;
    int who = 0;
    for (int k = 0; k < 8; ++k) {
      const float val = (float)x[vidx(2 * xx + (k & 1), 2 * yy + ((k >> 1) & 1), 2 * zz + (k >> 2), f) * ldx + c];
      if (val > best) {
        best = val;
        who = k;
      }
    }
    y[v * ldy + c] = (bf16)best;
    arg[e] = (uint8_t)who;
  }
}

__global__ void k_maxpool_backward(Grid g, int channels, const bf16 *dy, int ldy, const uint8_t *arg, bf16 *dx,
                                   int ldx, int accumulate) {
  // one thread per fine-grid element: each belongs to exactly one window
  const Grid f{2 * g.nx, 2 * g.ny, 2 * g.nz};
  const int64_t total = (int64_t)f.nx * f.ny * f.nz * channels;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % channels);
    const int64_t v = e / channels;
    const int xx = (int)(v % f.nx), yy = (int)((v / f.nx) % f.ny), zz = (int)(v / ((int64_t)f.nx * f.ny));
    const int k = (xx & 1) | ((yy & 1) << 1) | ((zz & 1) << 2);
    const int64_t cv = vidx(xx >> 1, yy >> 1, zz >> 1, g);
    const float routed = arg[cv * channels + c] == k ? (float)dy[cv * ldy + c] : 0.f;
    dx[v * ldx + c] = (bf16)(accumulate ? (float)dx[v * ldx + c] + routed : routed);
  }
}

// The same three operations on whole 8-channel groups (channels, strides and
// pointers multiples of 8 elements / 16 bytes, fewer than 2^31 groups): one
// thread per (voxel, group) with 16-byte loads and stores and 32-bit index
// arithmetic.  Thread e takes group q = e % groups of voxel e / groups.
__global__ void __launch_bounds__(256) k_maxpool8(Grid g, int groups, const bf16 *x, int ldx, bf16 *y, int ldy,
                                                  uint8_t *arg) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= g.nx * g.ny * g.nz * groups) return;
  const int q = e % groups, v = e / groups;
  const int cx = v % g.nx, cy = (v / g.nx) % g.ny, cz = v / (g.nx * g.ny);
  const Grid f{2 * g.nx, 2 * g.ny, 2 * g.nz};
  bf16x8 in[8];
#pragma unroll
  for (int k = 0; k < 8; ++k)
    in[k] = *reinterpret_cast<const bf16x8 *>(
        x + vidx(2 * cx + (k & 1), 2 * cy + ((k >> 1) & 1), 2 * cz + (k >> 2), f) * ldx + 8 * q);
  bf16x8 best;
  uint64_t who = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    float b = -INFINITY;
    int w = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {  // first strict maximum wins (NaN never does)
      const float val = (float)in[k][c];
      if (val > b) b = val, w = k;
    }
    best[c] = (bf16)b;
    who |= (uint64_t)w << (8 * c);
  }
  *reinterpret_cast<bf16x8 *>(y + (int64_t)v * ldy + 8 * q) = best;
  *reinterpret_cast<uint64_t *>(arg + (int64_t)v * (8 * groups) + 8 * q) = who;
}

__global__ void __launch_bounds__(256) k_maxpool_backward8(Grid g, int groups, const bf16 *dy, int ldy,
                                                           const uint8_t *arg, bf16 *dx, int ldx, int accumulate) {
  const Grid f{2 * g.nx, 2 * g.ny, 2 * g.nz};
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= f.nx * f.ny * f.nz * groups) return;
  const int q = e % groups, v = e / groups;
  const int xx = v % f.nx, yy = (v / f.nx) % f.ny, zz = v / (f.nx * f.ny);
  const int k = (xx & 1) | ((yy & 1) << 1) | ((zz & 1) << 2);
  const int64_t cv = vidx(xx >> 1, yy >> 1, zz >> 1, g);
  const uint64_t who = *reinterpret_cast<const uint64_t *>(arg + cv * (8 * groups) + 8 * q);
  const bf16x8 d = *reinterpret_cast<const bf16x8 *>(dy + cv * ldy + 8 * q);
  bf16 *out = dx + (int64_t)v * ldx + 8 * q;
  bf16x8 o = accumulate ? *reinterpret_cast<const bf16x8 *>(out) : bf16x8{};
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const float routed = (int)((who >> (8 * c)) & 0xff) == k ? (float)d[c] : 0.f;
    o[c] = (bf16)(accumulate ? (float)o[c] + routed : routed);
  }
  *reinterpret_cast<bf16x8 *>(out) = o;
}

__global__ void __launch_bounds__(256) k_relu_backward8(int n, int groups, const bf16 *y, int ldy, bf16 *dy,
                                                        int lddy) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n * groups) return;
  const int q = e % groups, row = e / groups;
  const bf16x8 yv = *reinterpret_cast<const bf16x8 *>(y + (int64_t)row * ldy + 8 * q);
  bf16 *p = dy + (int64_t)row * lddy + 8 * q;
  bf16x8 d = *reinterpret_cast<const bf16x8 *>(p);
#pragma unroll
  for (int c = 0; c < 8; ++c)
    if (!((float)yv[c] > 0.f)) d[c] = (bf16)0.f;
  *reinterpret_cast<bf16x8 *>(p) = d;
}

// whether an element-wise BF16 operation can run on whole 16-byte groups
bool groups8(int64_t elements_per_row, std::initializer_list<int64_t> strides,
             std::initializer_list<const void *> ptrs, int64_t rows) {
  if (elements_per_row % 8) return false;
  for (int64_t s : strides)
    if (s % 8) return false;
  for (const void *p : ptrs)
    if ((uintptr_t)p % 16) return false;
  return rows * (elements_per_row / 8) <= INT32_MAX - 255;
}

__global__ void k_relu_backward(int64_t n, int channels, const bf16 *y, int ldy, bf16 *dy, int lddy) {
  const int64_t total = n * channels;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e / channels;
    const int c = (int)(e % channels);
    if (!((float)y[row * ldy + c] > 0.f)) dy[row * lddy + c] = (bf16)0.f;
  }
}

__global__ void k_mse(int64_t n, int channels, const float *pred, const float *target, const uint8_t *mask, float scale,
                      bf16 *dpred, int ldd, float *loss) {
  __shared__ float red[256];
  float s = 0.f;
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n; row += (int64_t)gridDim.x * blockDim.x) {
    const bool on = mask[row] == 0;
    for (int c = 0; c < ldd; ++c) {
      float g = 0.f;
      if (c < channels && on) {
        const float d = pred[row * channels + c] - target[row * channels + c];
        s += d * d;
        g = scale * 2.f * d;
      }
      dpred[row * ldd + c] = (bf16)g;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, red[0]);
}

__global__ void k_adam(int64_t n, float *p, float *m, float *v, const float *g, bf16 *p16, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    const float pp = p[e] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    p[e] = pp;
    if (p16) p16[e] = (bf16)pp;
  }
}

// one voxel per thread: three 16-byte loads of y (12 FP32 channels), one
// 16-byte store of p
__global__ void __launch_bounds__(256) k_mix(int64_t n, const float *y, float d0, float d1, float d2, float *p) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const float4 *row = reinterpret_cast<const float4 *>(y + 12 * e);
  const float4 a = row[0], b = row[1], c = row[2];
  reinterpret_cast<float4 *>(p)[e] = make_float4(d0 * a.x + d1 * b.x + d2 * c.x, d0 * a.y + d1 * b.y + d2 * c.y,
                                                 d0 * a.z + d1 * b.z + d2 * c.z, d0 * a.w + d1 * b.w + d2 * c.w);
}

// one voxel per thread; dy rows (ldy a multiple of 8, 16-byte aligned) are
// written in 16-byte groups: channels 0..11 = d_j dp[k], the rest 0
__global__ void __launch_bounds__(256) k_mix_backward(int64_t n, const bf16 *dp, int ldp, float d0, float d1,
                                                      float d2, bf16 *dy, int ldy) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const float d[3] = {d0, d1, d2};
  float g[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) g[k] = (float)dp[e * ldp + k];
  bf16 *row = dy + e * ldy;
  for (int c0 = 0; c0 < ldy; c0 += 8) {
    bf16x8 o = {};
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (c0 + c < 12) o[c] = (bf16)(d[(c0 + c) / 4] * g[(c0 + c) % 4]);
    *reinterpret_cast<bf16x8 *>(row + c0) = o;
  }
}

__global__ void k_encode(int64_t n, const uint8_t *solid, float dx, float dy, float dz, bf16 *x) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const bool s = solid[e] != 0;
    bf16 *row = x + e * 8;
    row[0] = (bf16)(s ? 1.f : 0.f);
    row[1] = (bf16)(s ? 0.f : dx);
    row[2] = (bf16)(s ? 0.f : dy);
    row[3] = (bf16)(s ? 0.f : dz);
    for (int c = 4; c < 8; ++c) row[c] = (bf16)0.f;
  }
}

// ---- geometry input: distance to the nearest solid node -----------------------
// Shortest path along D3Q19 links (length 1 for faces, sqrt(2) for edges) to a
// solid node; each sweep is one Bellman-Ford relaxation d <- min(d, d(x+c) + |c|).
constexpr float kFar = 1e30f;

__global__ void k_dist_init(int64_t n, const uint8_t *solid, float *d) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    d[e] = solid[e] ? 0.f : kFar;
}

__global__ void __launch_bounds__(256) k_dist_sweep(Grid g, uint32_t periodic, const uint8_t *solid,
                                                    const float *din, float *dout) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  if (solid[e]) {
    dout[e] = 0.f;
    return;
  }
  const int x = (int)(e % g.nx), y = (int)((e / g.nx) % g.ny), z = (int)(e / ((int64_t)g.nx * g.ny));
  float best = din[e];
  lbm::static_for<19>([&](auto i) {
    constexpr int cx = lbm::D3Q19::C[i][0], cy = lbm::D3Q19::C[i][1], cz = lbm::D3Q19::C[i][2];
    if constexpr (cx != 0 || cy != 0 || cz != 0) {
      constexpr float len = ((cx != 0) + (cy != 0) + (cz != 0)) == 1 ? 1.0f : 1.41421356237309515f;
      int tx = x + cx, ty = y + cy, tz = z + cz;
      bool inside = true;
      if (tx < 0 || tx >= g.nx) {
        inside &= (periodic & 1u) != 0;
        tx = tx < 0 ? tx + g.nx : tx - g.nx;
      }
      if (ty < 0 || ty >= g.ny) {
        inside &= (periodic & 2u) != 0;
        ty = ty < 0 ? ty + g.ny : ty - g.ny;
      }
      if (tz < 0 || tz >= g.nz) {
        inside &= (periodic & 4u) != 0;
        tz = tz < 0 ? tz + g.nz : tz - g.nz;
      }
      if (inside) best = fminf(best, din[vidx(tx, ty, tz, g)] + len);
    }
  });
  dout[e] = best;
}

// x row = (solid, s, s^2, 0, ...) with s = min(d * scale, cap) on non-solid nodes
__global__ void k_encode_geometry(int64_t n, const uint8_t *solid, const float *d, float scale, float cap, bf16 *x) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const bool sd = solid[e] != 0;
    const float v = sd ? 0.f : fminf(d[e] * scale, cap);
    bf16 *row = x + e * 8;
    row[0] = (bf16)(sd ? 1.f : 0.f);
    row[1] = (bf16)v;
    row[2] = (bf16)(v * v);
    for (int c = 3; c < 8; ++c) row[c] = (bf16)0.f;
  }
}

__global__ void k_decode(int64_t n, const float *pred, const uint8_t *solid, double rho0, double scale, double *rho,
                         double *u, double *acc) {
  double s = 0.0, cnt = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const bool sd = solid[e] != 0;
    const double r = sd ? 0.0 : rho0 + scale * (double)pred[4 * e];
    rho[e] = r;
    for (int k = 0; k < 3; ++k) u[k * n + e] = sd ? 0.0 : scale * (double)pred[4 * e + 1 + k];
    if (!sd) {
      s += r;
      cnt += 1.0;
    }
  }
  if (acc) {
    atomicAdd(acc, s);
    atomicAdd(acc + 1, cnt);
  }
}

__global__ void k_renorm(int64_t n, const uint8_t *solid, double rho0, const double *acc, double *rho) {
  const double shift = acc[1] > 0.0 ? rho0 - acc[0] / acc[1] : 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    if (!solid[e]) rho[e] += shift;
}

__global__ void k_zero2(double *p) {
  if (threadIdx.x < 2) p[threadIdx.x] = 0.0;
}

unsigned grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

GemmArgs to_args(const lbm_nn_gemm *g) {
  GemmArgs a;
  a.rows = Grid{g->rows[0], g->rows[1], g->rows[2]};
  if (g->src_mode == LBM_NN_GATHER2)
    a.in_grid = Grid{2 * g->rows[0], 2 * g->rows[1], 2 * g->rows[2]};
  else
    a.in_grid = a.rows;
  if (g->dst_mode == LBM_NN_SCATTER2)
    a.out_grid = Grid{2 * g->rows[0], 2 * g->rows[1], 2 * g->rows[2]};
  else
    a.out_grid = a.rows;
  a.taps = g->taps;
  a.cin = g->cin;
  a.cout = g->cout;
  a.ldx = g->ldx;
  a.ldy = g->ldy;
  a.M = (int64_t)g->rows[0] * g->rows[1] * g->rows[2];
  a.x = static_cast<const bf16 *>(g->x);
  a.w = static_cast<const bf16 *>(g->w);
  a.bias = g->bias;
  a.y = g->y;
  a.gate = static_cast<const bf16 *>(g->gate);
  a.ldg = g->ldg;
  a.gate_ch = g->gate ? g->gate_channels : 0;
  return a;
}

int check_gemm(const lbm_nn_gemm *g, bool wgrad) {
  if (!g || !g->x || !g->y || (!wgrad && !g->w)) return set_error(LBM_ERR_ARG, "lbm_nn: NULL tensor");
  for (int k = 0; k < 3; ++k)
    if (g->rows[k] <= 0) return set_error(LBM_ERR_SHAPE, "lbm_nn: rows[%d] = %d", k, g->rows[k]);
  if ((int64_t)g->rows[0] * g->rows[1] * g->rows[2] > INT32_MAX)
    return set_error(LBM_ERR_SHAPE, "lbm_nn: more than 2^31 - 1 rows");
  const bool src_ok = g->src_mode == LBM_NN_IDENT || g->src_mode == LBM_NN_CONV3 || g->src_mode == LBM_NN_GATHER2;
  const bool dst_ok = g->dst_mode == LBM_NN_IDENT || g->dst_mode == LBM_NN_SCATTER2;
  if (!src_ok || !dst_ok) return set_error(LBM_ERR_ARG, "lbm_nn: modes %d/%d", g->src_mode, g->dst_mode);
  const int want_taps = g->src_mode == LBM_NN_CONV3 ? 27 : (g->src_mode == LBM_NN_GATHER2 ? 8 : 1);
  if (g->dst_mode == LBM_NN_SCATTER2 ? (g->taps != 8 || g->src_mode != LBM_NN_IDENT) : g->taps != want_taps)
    return set_error(LBM_ERR_ARG, "lbm_nn: %d taps for modes %d/%d", g->taps, g->src_mode, g->dst_mode);
  if (g->cin <= 0 || g->cin % 8 || g->ldx < g->cin || g->ldx % 8)
    return set_error(LBM_ERR_SHAPE, "lbm_nn: cin %d / ldx %d must be multiples of 8", g->cin, g->ldx);
  if (g->cout <= 0 || g->ldy < g->cout) return set_error(LBM_ERR_SHAPE, "lbm_nn: cout %d / ldy %d", g->cout, g->ldy);
  if ((!g->y_fp32 || wgrad) && (g->cout % 8 || g->ldy % 8))
    return set_error(LBM_ERR_SHAPE, "lbm_nn: BF16 rows need cout and ldy multiples of 8");
  if ((uintptr_t)g->x % 16 || (g->w && (uintptr_t)g->w % 16) || (uintptr_t)g->y % 16)
    return set_error(LBM_ERR_ARG, "lbm_nn: tensors must be 16-byte aligned");
  if (g->gate && !wgrad) {
    if (g->gate_channels <= 0 || g->gate_channels > g->cout || g->gate_channels % 8)
      return set_error(LBM_ERR_SHAPE, "lbm_nn: gate_channels %d (multiple of 8 in 8..cout = %d)", g->gate_channels,
                       g->cout);
    if (g->ldg < g->gate_channels || g->ldg % 8 || (uintptr_t)g->gate % 16)
      return set_error(LBM_ERR_SHAPE, "lbm_nn: gate rows need ldg %d >= gate_channels, a multiple of 8, 16-byte aligned",
                       g->ldg);
  }
  return LBM_OK;
}

#define NN_TRY(expr)                                                                                   \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ != hipSuccess) return set_error(LBM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));      \
  } while (0)

template <int SRC, int DST, int RF, bool F32, bool RELU>
hipError_t launch_fwd_rf(const GemmArgs &a, int nw, dim3 grid, float *part, int kper, hipStream_t s) {
  switch (nw) {
    case 1: hipLaunchKernelGGL((k_forward<SRC, DST, 1, RF, F32, RELU>), grid, dim3(256), 0, s, a, part, kper); break;
    case 2: hipLaunchKernelGGL((k_forward<SRC, DST, 2, RF, F32, RELU>), grid, dim3(256), 0, s, a, part, kper); break;
    case 3: hipLaunchKernelGGL((k_forward<SRC, DST, 3, RF, F32, RELU>), grid, dim3(256), 0, s, a, part, kper); break;
    default: hipLaunchKernelGGL((k_forward<SRC, DST, 4, RF, F32, RELU>), grid, dim3(256), 0, s, a, part, kper); break;
  }
  return hipGetLastError();
}

int fwd_nw(const GemmArgs &a) { return a.cout <= 16 ? 1 : (a.cout <= 32 ? 2 : (a.cout % 48 == 0 ? 3 : 4)); }

// Split-K plan of k_forward for small grids (fewer than 1024 blocks of 64 rows
// and at least 32 K steps of 32): S splits of kper (a multiple of 32) so that
// the launch has about 1024 blocks with at least 8 K steps each; S = 1: none.
// BF16 outputs with IDENT destinations only.
struct SplitPlan {
  int S, kper;
};
SplitPlan split_plan(const lbm_nn_gemm *g, const GemmArgs &a) {
  SplitPlan p{1, 0};
  if (g->y_fp32 || g->dst_mode != LBM_NN_IDENT) return p;
  const int nw = fwd_nw(a);
  const int64_t blocks = (a.M + 63) / 64 * ((a.cout + 16 * nw - 1) / (16 * nw));
  const int ksteps = (a.taps * a.cin + 31) / 32;
  if (blocks >= 1024 || ksteps < 32) return p;
  int S = (int)((1024 + blocks - 1) / blocks);
  if (S > ksteps / 8) S = ksteps / 8;
  if (S < 2) return p;
  const int per_steps = (ksteps + S - 1) / S;
  p.kper = 32 * per_steps;
  p.S = (ksteps + per_steps - 1) / per_steps;
  return p;
}

template <int SRC, int DST, bool F32, bool RELU>
hipError_t launch_fwd(const GemmArgs &a, hipStream_t s, const SplitPlan &sp = SplitPlan{1, 0}, float *part = nullptr) {
  const int nw = fwd_nw(a);
  const unsigned gy = (unsigned)((a.cout + 16 * nw - 1) / (16 * nw));
  if constexpr (DST == LBM_NN_IDENT && !F32) {
    if (sp.S > 1) {
      hipError_t e = launch_fwd_rf<SRC, DST, 1, F32, RELU>(a, nw, dim3((unsigned)((a.M + 63) / 64), gy, sp.S), part,
                                                           sp.kper, s);
      if (e != hipSuccess) return e;
      const int64_t n = a.M * (a.cout / 8);
      hipLaunchKernelGGL(k_forward_finish<RELU>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a,
                         (const float *)part, sp.S);
      return hipGetLastError();
    }
  }
  // 256 rows per block where that still gives the device >= 512 blocks, else 64
  const int64_t big = (a.M + 255) / 256 * gy;
  if constexpr (DST == LBM_NN_SCATTER2 && !F32) {
    const int ks = (a.cin + 31) / 32;
    const int rf = big >= 512 && ks <= 2 ? 4 : 1;
    const size_t lds = (size_t)(2 * 16 * nw * (32 * ks + 8) + 64 * rf * (16 * nw + 8)) * 2;
    if (ks <= 8 / rf && lds <= 65536) {
      const int64_t blocks = (a.M + 64 * rf - 1) / (64 * rf) * gy;
      unsigned tz = 1;
      while (blocks * tz < 512 && tz < 8) tz *= 2;
      const dim3 grid((unsigned)((a.M + 64 * rf - 1) / (64 * rf)), gy, tz);
      if (rf == 4) {
        switch (nw) {
          case 1: return launch_up2_nw<1, 4>(a, RELU, grid, lds, s);
          case 2: return launch_up2_nw<2, 4>(a, RELU, grid, lds, s);
          case 3: return launch_up2_nw<3, 4>(a, RELU, grid, lds, s);
          default: return launch_up2_nw<4, 4>(a, RELU, grid, lds, s);
        }
      }
      switch (nw) {
        case 1: return launch_up2_nw<1, 1>(a, RELU, grid, lds, s);
        case 2: return launch_up2_nw<2, 1>(a, RELU, grid, lds, s);
        case 3: return launch_up2_nw<3, 1>(a, RELU, grid, lds, s);
        default: return launch_up2_nw<4, 1>(a, RELU, grid, lds, s);
      }
    }
  }
  if (big >= 512)
    return launch_fwd_rf<SRC, DST, 4, F32, RELU>(a, nw, dim3((unsigned)((a.M + 255) / 256), gy), nullptr, 0, s);
  return launch_fwd_rf<SRC, DST, 1, F32, RELU>(a, nw, dim3((unsigned)((a.M + 63) / 64), gy), nullptr, 0, s);
}

template <int NW, int CC>
hipError_t launch_brick_cc(const GemmArgs &a, bool relu, dim3 grid, hipStream_t s) {
  const size_t dyn = brick_dyn<NW, CC>() ? 2 * (size_t)brick_lds<NW, CC>() : 0;
  const void *k = relu ? reinterpret_cast<const void *>(&k_conv3_brick<NW, CC, true>)
                       : reinterpret_cast<const void *>(&k_conv3_brick<NW, CC, false>);
  if (dyn) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    if (e != hipSuccess) return e;
  }
  if (relu)
    hipLaunchKernelGGL((k_conv3_brick<NW, CC, true>), grid, dim3(256), dyn, s, a);
  else
    hipLaunchKernelGGL((k_conv3_brick<NW, CC, false>), grid, dim3(256), dyn, s, a);
  return hipGetLastError();
}

template <int NW>
hipError_t launch_brick_nw(const GemmArgs &a, int cc, bool relu, dim3 grid, hipStream_t s) {
  switch (cc) {
    case 8: return launch_brick_cc<NW, 8>(a, relu, grid, s);
    case 24: return launch_brick_cc<NW, 24>(a, relu, grid, s);
    case 48: return launch_brick_cc<NW, 48>(a, relu, grid, s);
    default: return launch_brick_cc<NW, 32>(a, relu, grid, s);
  }
}

// The brick kernel for a 3x3x3 convolution with BF16 output: channel chunks of
// 8 (an 8-channel input), 24 or 48 (the whole input: one halo staging per block;
// the 48-channel halo takes 69 KB of dynamic LDS, two blocks per CU) or 32
// (multiples of 32), and enough bricks to fill the device; returns false to use
// k_forward instead.
// channel chunk of the brick kernel for a 3x3x3 convolution with BF16
// output, or 0 where it does not apply (an unsupported input width, a grid
// thinner than a brick, whose halo would wrap past one period, or too few
// bricks to fill the device)
int brick_chunk(const GemmArgs &a, bool f32) {
  if (f32) return 0;
  int cc;
  if (a.cin == 8)
    cc = 8;
  else if (a.cin == 24 || a.cin == 48)
    cc = a.cin;
  else if (a.cin % 32 == 0)
    cc = 32;
  else
    return 0;
  if (a.rows.nx < kBrickX || a.rows.ny < kBrickY || a.rows.nz < kBrickZ) return 0;
  const int nw = fwd_nw(a);
  const int64_t bricks = (int64_t)((a.rows.nx + kBrickX - 1) / kBrickX) * ((a.rows.ny + kBrickY - 1) / kBrickY) *
                         ((a.rows.nz + kBrickZ - 1) / kBrickZ);
  if (bricks * ((a.cout + 16 * nw - 1) / (16 * nw)) < 256) return 0;
  return cc;
}

bool try_brick(const GemmArgs &a, bool f32, bool relu, hipStream_t s, hipError_t *err) {
  const int cc = brick_chunk(a, f32);
  if (!cc) return false;
  const int nw = fwd_nw(a);
  const int64_t bricks = (int64_t)((a.rows.nx + kBrickX - 1) / kBrickX) * ((a.rows.ny + kBrickY - 1) / kBrickY) *
                         ((a.rows.nz + kBrickZ - 1) / kBrickZ);
  const dim3 grid((unsigned)bricks, (unsigned)((a.cout + 16 * nw - 1) / (16 * nw)), 1);
  switch (nw) {
    case 1: *err = launch_brick_nw<1>(a, cc, relu, grid, s); break;
    case 2: *err = launch_brick_nw<2>(a, cc, relu, grid, s); break;
    case 3: *err = launch_brick_nw<3>(a, cc, relu, grid, s); break;
    default: *err = launch_brick_nw<4>(a, cc, relu, grid, s); break;
  }
  return true;
}

template <int SRC, int DST>
hipError_t fwd_act(const GemmArgs &a, bool f32, bool relu, const SplitPlan &sp, float *part, hipStream_t s) {
  if constexpr (SRC == LBM_NN_CONV3 && DST == LBM_NN_IDENT) {
    hipError_t e = hipSuccess;
    if (try_brick(a, f32, relu, s, &e)) return e;
  }
  if (f32) return relu ? launch_fwd<SRC, DST, true, true>(a, s) : launch_fwd<SRC, DST, true, false>(a, s);
  return relu ? launch_fwd<SRC, DST, false, true>(a, s, sp, part) : launch_fwd<SRC, DST, false, false>(a, s, sp, part);
}

// whether lbm_nn_forward takes the brick kernel for this layer (no workspace then)
bool takes_brick(const lbm_nn_gemm *g, const GemmArgs &a) {
  return g->src_mode == LBM_NN_CONV3 && g->dst_mode == LBM_NN_IDENT && brick_chunk(a, g->y_fp32 != 0) != 0;
}

// workspace floats of lbm_nn_forward_ws (the split-K partial sums; 0: none)
int64_t fwd_ws_floats(const lbm_nn_gemm *g, const GemmArgs &a) {
  if (takes_brick(g, a)) return 0;
  const SplitPlan sp = split_plan(g, a);
  return sp.S > 1 ? (int64_t)sp.S * a.M * a.cout : 0;
}

// Grid of k_wgrad: (voxel chunks, taps * cblocks, nblocks), about 2048 blocks
// with chunks of a multiple of 128 voxels.
struct GenericWgradGrid {
  int cblocks, nblocks;
  int64_t chunk, chunks;
};
GenericWgradGrid generic_wgrad_grid(const GemmArgs &a, int cf, int nf) {
  GenericWgradGrid w;
  w.cblocks = (a.cin + 16 * cf - 1) / (16 * cf);
  w.nblocks = (a.cout + 16 * nf - 1) / (16 * nf);
  const int64_t other = (int64_t)a.taps * w.cblocks * w.nblocks;
  int64_t chunks = (2048 + other - 1) / other;
  const int64_t max_chunks = (a.M + 127) / 128;
  if (chunks > max_chunks) chunks = max_chunks;
  if (chunks < 1) chunks = 1;
  int64_t chunk = (a.M + chunks - 1) / chunks;
  w.chunk = (chunk + 127) / 128 * 128;
  w.chunks = (a.M + w.chunk - 1) / w.chunk;
  return w;
}
void generic_wgrad_frags(const GemmArgs &a, int *cf, int *nf) {
  *cf = a.cin <= 16 ? 1 : 2;
  *nf = a.cout <= 16 ? 1 : 2;
}
int64_t generic_wgrad_ws_floats(const GemmArgs &a) {
  int cf, nf;
  generic_wgrad_frags(a, &cf, &nf);
  const GenericWgradGrid w = generic_wgrad_grid(a, cf, nf);
  return w.chunks * a.taps * w.cblocks * w.nblocks * 256 * cf * nf;
}

template <int SRC, int DST, int CF, int NF>
hipError_t launch_wgrad_cf(const GemmArgs &a, float *dw, float *ws, float *db, hipStream_t s) {
  const GenericWgradGrid w = generic_wgrad_grid(a, CF, NF);
  hipLaunchKernelGGL((k_wgrad<SRC, DST, CF, NF>), dim3((unsigned)w.chunks, (unsigned)(a.taps * w.cblocks),
                                                       (unsigned)w.nblocks),
                     dim3(256), 0, s, a, dw, w.chunk, w.cblocks, ws, db);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !ws) return e;
  return launch_wgrad_sum(ws, w.chunks, (int64_t)a.taps * w.cblocks * w.nblocks, CF, NF, w.cblocks, 1, a.taps, a.cin,
                          a.cout, dw, s);
}

// Grid of the brick weight gradient: about two blocks per compute unit in
// all; each block sums its bricks in registers.
struct WgradGrid {
  int cblocks, nblocks;
  int64_t per, gx;
};
WgradGrid wgrad_grid(const GemmArgs &a, int cf, int nf) {
  WgradGrid w;
  w.cblocks = (a.cin + 16 * cf - 1) / (16 * cf);
  w.nblocks = (a.cout + 16 * nf - 1) / (16 * nf);
  const int64_t nbricks = (int64_t)((a.rows.nx + kWbX - 1) / kWbX) * ((a.rows.ny + kWbY - 1) / kWbY) *
                          ((a.rows.nz + kWbZ - 1) / kWbZ);
  const int64_t tiles = (int64_t)w.cblocks * w.nblocks;
  w.per = (nbricks * tiles + 511) / 512;
  if (w.per < 1) w.per = 1;
  w.gx = (nbricks + w.per - 1) / w.per;
  return w;
}

template <int CF, int NF>
hipError_t launch_wgrad_brick_cf(const GemmArgs &a, float *dw, float *ws, float *db, hipStream_t s) {
  using WB = WBrick<CF, NF>;
  const WgradGrid w = wgrad_grid(a, CF, NF);
  const int tiles = w.cblocks * w.nblocks;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_wgrad_brick<CF, NF>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, WB::LDS);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_wgrad_brick<CF, NF>), dim3((unsigned)w.gx, (unsigned)tiles), dim3(WB::T), WB::LDS, s, a, dw,
                     (int)w.per, w.cblocks, ws, db);
  e = hipGetLastError();
  if (e != hipSuccess || !ws) return e;
  return launch_wgrad_sum(ws, w.gx, tiles, CF, NF, w.cblocks, 27, 27, a.cin, a.cout, dw, s);
}

// channel tile width (in 16-channel fragments, 1..3) that pads c channels least
int wgrad_frags(int c, int max_frags) {
  int best = 1, waste = 1 << 30;
  for (int f = 1; f <= max_frags; ++f) {
    const int w = (c + 16 * f - 1) / (16 * f) * 16 * f - c;
    if (w <= waste) best = f, waste = w;
  }
  return best;
}

void wgrad_brick_frags(const GemmArgs &a, int *cf, int *nf) {
  *cf = wgrad_frags(a.cin, 3);
  *nf = wgrad_frags(a.cout, *cf == 3 ? 2 : 3);
}

// The brick weight gradient for 3x3x3 convolutions: with a workspace on any
// grid that gives at least 128 (brick run, channel tile) blocks, without one
// (FP32 atomics, whose contention grows with the block count) on grids of at
// least 2048 bricks of 8x4x4.  The halo's periodic wrap needs the grid to be
// at least one brick along every axis.
bool wgrad_brick_applies(const GemmArgs &a, bool with_ws) {
  if (a.rows.nx < kWbX || a.rows.ny < kWbY || a.rows.nz < kWbZ) return false;
  const int64_t nbricks = (int64_t)((a.rows.nx + kWbX - 1) / kWbX) * ((a.rows.ny + kWbY - 1) / kWbY) *
                          ((a.rows.nz + kWbZ - 1) / kWbZ);
  if (!with_ws) return nbricks >= 2048;
  int cf, nf;
  wgrad_brick_frags(a, &cf, &nf);
  const WgradGrid w = wgrad_grid(a, cf, nf);
  return w.gx * w.cblocks * w.nblocks >= 128;
}
// Workspace floats the brick weight gradient's partial sums need (0 when the
// brick kernel does not apply).
int64_t wgrad_brick_ws_floats(const GemmArgs &a) {
  if (!wgrad_brick_applies(a, true)) return 0;
  int cf, nf;
  wgrad_brick_frags(a, &cf, &nf);
  const WgradGrid w = wgrad_grid(a, cf, nf);
  return (int64_t)w.cblocks * w.nblocks * w.gx * 27 * 256 * cf * nf;
}

// Runs the brick weight gradient if it applies (returns false to use k_wgrad
// instead); ws: partial sums (wgrad_brick_ws_floats) or NULL for atomics; db:
// the bias gradient, accumulated from the staged dy tiles (one atomic add per
// block and channel), or NULL.
bool try_wgrad_brick(const GemmArgs &a, float *dw, float *ws, float *db, hipStream_t s, hipError_t *err) {
  if (!wgrad_brick_applies(a, ws != nullptr)) return false;
  int cf, nf;
  wgrad_brick_frags(a, &cf, &nf);
  switch (cf * 4 + nf) {
    case 5: *err = launch_wgrad_brick_cf<1, 1>(a, dw, ws, db, s); break;
    case 6: *err = launch_wgrad_brick_cf<1, 2>(a, dw, ws, db, s); break;
    case 7: *err = launch_wgrad_brick_cf<1, 3>(a, dw, ws, db, s); break;
    case 9: *err = launch_wgrad_brick_cf<2, 1>(a, dw, ws, db, s); break;
    case 10: *err = launch_wgrad_brick_cf<2, 2>(a, dw, ws, db, s); break;
    case 11: *err = launch_wgrad_brick_cf<2, 3>(a, dw, ws, db, s); break;
    case 13: *err = launch_wgrad_brick_cf<3, 1>(a, dw, ws, db, s); break;
    default: *err = launch_wgrad_brick_cf<3, 2>(a, dw, ws, db, s); break;
  }
  return true;
}

// Grid of k_wgrad_up2: chunks of 64-row multiples x channel tiles, about 512 blocks.
struct Up2WgradGrid {
  int cf, nf, cblocks, nblocks, chunk, chunks;
};
Up2WgradGrid up2_wgrad_grid(const GemmArgs &a) {
  Up2WgradGrid w;
  w.cf = wgrad_frags(a.cin, 3);
  w.nf = wgrad_frags(a.cout, w.cf == 3 ? 2 : 3);
  w.cblocks = (a.cin + 16 * w.cf - 1) / (16 * w.cf);
  w.nblocks = (a.cout + 16 * w.nf - 1) / (16 * w.nf);
  const int64_t tiles = (int64_t)w.cblocks * w.nblocks;
  int64_t chunks = (512 + tiles - 1) / tiles;
  int64_t chunk = (a.M + chunks - 1) / chunks;
  chunk = (chunk + 63) / 64 * 64;
  w.chunk = (int)chunk;
  w.chunks = (int)((a.M + chunk - 1) / chunk);
  return w;
}
int64_t up2_wgrad_ws_floats(const GemmArgs &a) {
  const Up2WgradGrid w = up2_wgrad_grid(a);
  return (int64_t)w.cblocks * w.nblocks * w.chunks * 8 * 256 * w.cf * w.nf;
}
template <int CF, int NF>
hipError_t launch_wgrad_up2_cf(const GemmArgs &a, const Up2WgradGrid &w, float *dw, float *ws, float *db,
                               hipStream_t s) {
  const int tiles = w.cblocks * w.nblocks;
  hipLaunchKernelGGL((k_wgrad_up2<CF, NF>), dim3((unsigned)w.chunks, (unsigned)tiles), dim3(512), 0, s, a, dw, w.chunk,
                     w.cblocks, ws, db);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !ws) return e;
  return launch_wgrad_sum(ws, w.chunks, tiles, CF, NF, w.cblocks, 8, 8, a.cin, a.cout, dw, s);
}
hipError_t launch_wgrad_up2(const GemmArgs &a, float *dw, float *ws, float *db, hipStream_t s) {
  const Up2WgradGrid w = up2_wgrad_grid(a);
  switch (w.cf * 4 + w.nf) {
    case 5: return launch_wgrad_up2_cf<1, 1>(a, w, dw, ws, db, s);
    case 6: return launch_wgrad_up2_cf<1, 2>(a, w, dw, ws, db, s);
    case 7: return launch_wgrad_up2_cf<1, 3>(a, w, dw, ws, db, s);
    case 9: return launch_wgrad_up2_cf<2, 1>(a, w, dw, ws, db, s);
    case 10: return launch_wgrad_up2_cf<2, 2>(a, w, dw, ws, db, s);
    case 11: return launch_wgrad_up2_cf<2, 3>(a, w, dw, ws, db, s);
    case 13: return launch_wgrad_up2_cf<3, 1>(a, w, dw, ws, db, s);
    default: return launch_wgrad_up2_cf<3, 2>(a, w, dw, ws, db, s);
  }
}

// the generic weight gradient; db (or NULL): the bias gradient, summed in the same kernel
template <int SRC, int DST>
hipError_t launch_wgrad(const GemmArgs &a, float *dw, float *ws, float *db, hipStream_t s) {
  int cf, nf;
  generic_wgrad_frags(a, &cf, &nf);
  if (cf == 1 && nf == 1) return launch_wgrad_cf<SRC, DST, 1, 1>(a, dw, ws, db, s);
  if (cf == 1) return launch_wgrad_cf<SRC, DST, 1, 2>(a, dw, ws, db, s);
  if (nf == 1) return launch_wgrad_cf<SRC, DST, 2, 1>(a, dw, ws, db, s);
  return launch_wgrad_cf<SRC, DST, 2, 2>(a, dw, ws, db, s);
}

// workspace floats of lbm_nn_wgrad_ws for a layer (the brick kernel's where it applies)
int64_t wgrad_ws_floats(const lbm_nn_gemm *g, const GemmArgs &a) {
  if (g->src_mode == LBM_NN_CONV3 && g->dst_mode == LBM_NN_IDENT && wgrad_brick_applies(a, true))
    return wgrad_brick_ws_floats(a);
  if (g->dst_mode == LBM_NN_SCATTER2) return up2_wgrad_ws_floats(a);
  return generic_wgrad_ws_floats(a);
}

}  // namespace
}  // namespace nn
}  // namespace lbm

using namespace lbm::nn;
using lbm::set_error;

static int forward_impl(const lbm_nn_gemm *g, float *ws, int64_t ws_floats, void *stream) {
  int rc = check_gemm(g, false);
  if (rc) return rc;
  const GemmArgs a = to_args(g);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool f32 = g->y_fp32 != 0, relu = g->relu != 0;
  SplitPlan sp{1, 0};
  if (ws) {
    const int64_t need = fwd_ws_floats(g, a);
    if (ws_floats < need)
      return set_error(LBM_ERR_ARG, "lbm_nn_forward_ws: workspace of %lld floats, %lld needed", (long long)ws_floats,
                       (long long)need);
    if (need > 0) sp = split_plan(g, a);
  }
  if (g->dst_mode == LBM_NN_SCATTER2) {
    NN_TRY((fwd_act<LBM_NN_IDENT, LBM_NN_SCATTER2>(a, f32, relu, sp, ws, s)));
  } else if (g->src_mode == LBM_NN_CONV3) {
    NN_TRY((fwd_act<LBM_NN_CONV3, LBM_NN_IDENT>(a, f32, relu, sp, ws, s)));
  } else if (g->src_mode == LBM_NN_GATHER2) {
    NN_TRY((fwd_act<LBM_NN_GATHER2, LBM_NN_IDENT>(a, f32, relu, sp, ws, s)));
  } else {
    NN_TRY((fwd_act<LBM_NN_IDENT, LBM_NN_IDENT>(a, f32, relu, sp, ws, s)));
  }
  return LBM_OK;
}

extern "C" int lbm_nn_forward(const lbm_nn_gemm *g, void *stream) { return forward_impl(g, nullptr, 0, stream); }

extern "C" int lbm_nn_forward_ws(const lbm_nn_gemm *g, float *ws, int64_t ws_floats, void *stream) {
  return forward_impl(g, ws, ws_floats, stream);
}

extern "C" int64_t lbm_nn_forward_workspace(const lbm_nn_gemm *g) {
  if (check_gemm(g, false)) return -1;
  return fwd_ws_floats(g, to_args(g));
}

// Weight gradient with an optional workspace for the brick kernel's partial sums.
static int wgrad_impl(const lbm_nn_gemm *g, float *dw, float *db, float *ws, int64_t ws_floats, void *stream) {
  int rc = check_gemm(g, true);
  if (rc) return rc;
  if (!dw) return set_error(LBM_ERR_ARG, "lbm_nn_wgrad: NULL dw");
  if (ws) {
    const int64_t need = wgrad_ws_floats(g, to_args(g));
    if (ws_floats < need)
      return set_error(LBM_ERR_ARG, "lbm_nn_wgrad_ws: workspace of %lld floats, %lld needed", (long long)ws_floats,
                       (long long)need);
  }
  const GemmArgs a = to_args(g);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the bias gradient is summed inside the weight-gradient kernels
  if (g->dst_mode == LBM_NN_SCATTER2) {
    NN_TRY(launch_wgrad_up2(a, dw, ws, db, s));
  } else if (g->src_mode == LBM_NN_CONV3) {
    hipError_t e = hipSuccess;
    if (!try_wgrad_brick(a, dw, ws, db, s, &e)) e = launch_wgrad<LBM_NN_CONV3, LBM_NN_IDENT>(a, dw, ws, db, s);
    NN_TRY(e);
  } else if (g->src_mode == LBM_NN_GATHER2) {
    NN_TRY((launch_wgrad<LBM_NN_GATHER2, LBM_NN_IDENT>(a, dw, ws, db, s)));
  } else {
    NN_TRY((launch_wgrad<LBM_NN_IDENT, LBM_NN_IDENT>(a, dw, ws, db, s)));
  }
  return LBM_OK;
}

extern "C" int lbm_nn_wgrad(const lbm_nn_gemm *g, float *dw, float *db, void *stream) {
  return wgrad_impl(g, dw, db, nullptr, 0, stream);
}

extern "C" int64_t lbm_nn_wgrad_workspace(const lbm_nn_gemm *g) {
  if (check_gemm(g, true)) return -1;
  return wgrad_ws_floats(g, to_args(g));
}

extern "C" int lbm_nn_wgrad_ws(const lbm_nn_gemm *g, float *dw, float *db, float *ws, int64_t ws_floats,
                               void *stream) {
  return wgrad_impl(g, dw, db, ws, ws_floats, stream);
}

extern "C" int lbm_nn_backward_weights_batch(int32_t count, const lbm_nn_wt_job *jobs, void *stream) {
  if (count < 0 || count > LBM_NN_WT_JOBS_MAX || (count > 0 && !jobs))
    return set_error(LBM_ERR_ARG, "lbm_nn_backward_weights_batch: %d jobs (at most %d)", count, LBM_NN_WT_JOBS_MAX);
  WtJobs J{};
  int64_t blocks = 0;
  for (int j = 0; j < count; ++j) {
    const lbm_nn_wt_job &b = jobs[j];
    if (!b.w || !b.wt || b.taps <= 0 || b.cin <= 0 || b.cout <= 0 ||
        (b.mode != LBM_NN_CONV3 && b.mode != LBM_NN_SCATTER2 && b.mode != LBM_NN_IDENT) ||
        (b.mode == LBM_NN_CONV3 && b.taps != 27))
      return set_error(LBM_ERR_ARG, "lbm_nn_backward_weights_batch: job %d", j);
    J.job[j] = b;
    J.first[j] = (int)blocks;
    blocks += ((int64_t)b.taps * b.cin * b.cout + 255) / 256;
    if (blocks > INT32_MAX) return set_error(LBM_ERR_SHAPE, "lbm_nn_backward_weights_batch: too many weights");
  }
  J.first[count] = (int)blocks;
  J.count = count;
  if (blocks == 0) return LBM_OK;
  hipLaunchKernelGGL(k_backward_weights_batch, dim3((unsigned)blocks), dim3(256), 0, static_cast<hipStream_t>(stream), J);
  NN_TRY(hipGetLastError());
  return LBM_OK;
}

extern "C" int lbm_nn_backward_weights(int32_t mode, int32_t taps, int32_t cin, int32_t cout, const void *w, void *wt,
                                       void *stream) {
  if (!w || !wt || taps <= 0 || cin <= 0 || cout <= 0) return set_error(LBM_ERR_ARG, "lbm_nn_backward_weights: args");
  if (mode == LBM_NN_CONV3 && taps != 27) return set_error(LBM_ERR_ARG, "lbm_nn_backward_weights: CONV3 needs 27 taps");
  const int64_t n = (int64_t)taps * cin * cout;
  hipLaunchKernelGGL(k_backward_weights, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), mode, taps,
                     cin, cout, static_cast<const bf16 *>(w), static_cast<bf16 *>(wt));
  NN_TRY(hipGetLastError());
  return LBM_OK;
}

extern "C" int lbm_nn_maxpool2(const int32_t grid[3], int32_t channels, const void *x, int32_t ldx, void *y,
                               int32_t ldy, uint8_t *arg, void *stream) {
  if (!grid || !x || !y || !arg || channels <= 0 || ldx < channels || ldy < channels)
    return set_error(LBM_ERR_ARG, "lbm_nn_maxpool2: args");
  const Grid g{grid[0], grid[1], grid[2]};
  const int64_t n = (int64_t)g.nx * g.ny * g.nz * channels;
  if (n == 0) return LBM_OK;
  if (groups8(channels, {ldx, ldy}, {x, y}, 8 * (int64_t)g.nx * g.ny * g.nz) && (uintptr_t)arg % 8 == 0) {
    hipLaunchKernelGGL(k_maxpool8, dim3((unsigned)((n / 8 + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), g, channels / 8, static_cast<const bf16 *>(x), ldx,
                       static_cast<bf16 *>(y), ldy, arg);
    NN_TRY(hipGetLastError());
    return LBM_OK;
  }
  hipLaunchKernelGGL(k_maxpool, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), g, channels,
                     static_cast<const bf16 *>(x), ldx, static_cast<bf16 *>(y), ldy, arg);
  NN_TRY(hipGetLastError());
  return LBM_OK;
}

extern "C" int lbm_nn_maxpool2_backward(const int32_t grid[3], int32_t channels, const void *dy, int32_t ldy,
                                        const uint8_t *arg, void *dx, int32_t ldx, int32_t accumulate, void *stream) {
  if (!grid || !dy || !dx || !arg || channels <= 0 || ldx < channels || ldy < channels)
    return set_error(LBM_ERR_ARG, "lbm_nn_maxpool2_backward: args");
  const Grid g{grid[0], grid[1], grid[2]};
  const int64_t n = (int64_t)8 * g.nx * g.ny * g.nz * channels;
  if (n == 0) return LBM_OK;
  if (groups8(channels, {ldx, ldy}, {dx, dy}, 8 * (int64_t)g.nx * g.ny * g.nz) && (uintptr_t)arg % 8 == 0) {
    hipLaunchKernelGGL(k_maxpool_backward8, dim3((unsigned)((n / 8 + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), g, channels / 8, static_cast<const bf16 *>(dy), ldy, arg,
                       static_cast<bf16 *>(dx), ldx, accumulate);
    NN_TRY(hipGetLastError());
    return LBM_OK;
  }
  hipLaunchKernelGGL(k_maxpool_backward, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), g,
                     channels, static_cast<const bf16 *>(dy), ldy, arg, static_cast<bf16 *>(dx), ldx, accumulate);
  NN_TRY(hipGetLastError());
  return LBM_OK;
}

extern "C" int lbm_nn_relu_backward(int64_t n, int32_t channels, const void *y, int32_t ld_y, void *dy, int32_t ld_dy,
                                    void *stream) {
  if (!y || !dy || n < 0 || channels <= 0) return set_error(LBM_ERR_ARG, "lbm_nn_relu_backward: args");
  if (n == 0) return LBM_OK;
  if (groups8(channels, {ld_y, ld_dy}, {y, dy}, n)) {
    hipLaunchKernelGGL(k_relu_backward8, dim3((unsigned)((n * (channels / 8) + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), (int)n, channels / 8, static_cast<const bf16 *>(y), ld_y,
                       static_cast<bf16 *>(dy), ld_dy);
    NN_TRY(hipGetLastError());
    return LBM_OK;
  }
  hipLaunchKernelGGL(k_relu_backward, dim3(grid_for(n * channels)), dim3(256), 0, static_cast<hipStream_t>(stream), n,
                     channels, static_cast<const bf16 *>(y), ld_y, static_cast<bf16 *>(dy), ld_dy);
  NN_TRY(hipGetLastError());
  return LBM_OK;
}

extern "C" int lbm_nn_mse(int64_t n, int32_t channels, const float *pred, const float *target, const uint8_t *mask,
                          float scale, void *dpred, int32_t ldd, float *loss_acc, void *stream) {
  if (!pred || !target || !mask || !dpred || !loss_acc || channels <= 0 || ldd < channels)
    return set_error(LBM_ERR_ARG, "lbm_nn_mse: args");
  hipLaunchKernelGGL(k_mse, dim3(grid_for(n) < 2048 ? grid_for(n) : 2048), dim3(256), 0,
                     static_cast<hipStream_t>(stream), n, channels, pred, target, mask, scale,
                     static_cast<bf16 *>(dpred), ldd, loss_acc);
  NN_TRY(hipGetLastError());
  return LBM_OK;
}

extern "C" int lbm_nn_adam(int64_t n, float *p, float *m, float *v, const float *g, void *p16, float lr, float beta1,
                           float beta2, float eps, int32_t step, void *stream) {
  if (!p || !m || !v || !g || n < 0 || step < 1) return set_error(LBM_ERR_ARG, "lbm_nn_adam: args");
  const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), n, p, m, v, g,
                     static_cast<bf16 *>(p16), lr, beta1, beta2, eps, c1, c2);
  NN_TRY(hipGetLastError());
  return LBM_OK;
}

extern "C" int lbm_nn_mix(int64_t n, const float *y, const float dir[3], float *p, void *stream) {
  if (!y || !dir || !p || n < 0) return set_error(LBM_ERR_ARG, "lbm_nn_mix: args");
  if ((uintptr_t)y % 16 || (uintptr_t)p % 16) return set_error(LBM_ERR_ARG, "lbm_nn_mix: y and p must be 16-byte aligned");
  if (n == 0) return LBM_OK;
  if (n > (int64_t)INT32_MAX * 256) return set_error(LBM_ERR_SHAPE, "lbm_nn_mix: too many nodes");
  hipLaunchKernelGGL(k_mix, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream), n, y, dir[0], dir[1],
                     dir[2], p);
  NN_TRY(hipGetLastError());
  return LBM_OK;
}

extern "C" int lbm_nn_mix_backward(int64_t n, const void *dp, int32_t ldp, const float dir[3], void *dy, int32_t ldy,
                                   void *stream) {
  if (!dp || !dir || !dy || n < 0 || ldp < 4 || ldy < 12) return set_error(LBM_ERR_ARG, "lbm_nn_mix_backward: args");
  if (ldy % 8 || (uintptr_t)dy % 16) return set_error(LBM_ERR_ARG, "lbm_nn_mix_backward: dy rows need ldy % 8 == 0, 16-byte aligned");
  if (n == 0) return LBM_OK;
  if (n > (int64_t)INT32_MAX * 256) return set_error(LBM_ERR_SHAPE, "lbm_nn_mix_backward: too many nodes");
  hipLaunchKernelGGL(k_mix_backward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream), n,
                     static_cast<const bf16 *>(dp), ldp, dir[0], dir[1], dir[2], static_cast<bf16 *>(dy), ldy);
  NN_TRY(hipGetLastError());
  return LBM_OK;
}

extern "C" int lbm_nn_encode_input(int64_t n, const uint8_t *solid, const float dir[3], void *x, void *stream) {
  if (!solid || !dir || !x || n < 0) return set_error(LBM_ERR_ARG, "lbm_nn_encode_input: args");
  hipLaunchKernelGGL(k_encode, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), n, solid, dir[0],
                     dir[1], dir[2], static_cast<bf16 *>(x));
  NN_TRY(hipGetLastError());
  return LBM_OK;
}

extern "C" int lbm_nn_distance(const int32_t shape[3], uint32_t periodic, const uint8_t *solid, int32_t sweeps,
                               float *dist, float *tmp, void *stream) {
  if (!shape || !solid || !dist || !tmp || dist == tmp) return set_error(LBM_ERR_ARG, "lbm_nn_distance: args");
  if (shape[0] <= 0 || shape[1] <= 0 || shape[2] <= 0 || periodic > 7u || sweeps < 0 || sweeps > 100000)
    return set_error(LBM_ERR_ARG, "lbm_nn_distance: shape %d x %d x %d, periodic %u, sweeps %d", shape[0], shape[1],
                     shape[2], periodic, sweeps);
  const Grid g{shape[0], shape[1], shape[2]};
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_dist_init, dim3(grid_for(n)), dim3(256), 0, s, n, solid, dist);
  const unsigned grid = (unsigned)((n + 255) / 256);
  for (int k = 0; k < (sweeps + 1) / 2; ++k) {  // pairs of sweeps end in dist
    hipLaunchKernelGGL(k_dist_sweep, dim3(grid), dim3(256), 0, s, g, periodic, solid, (const float *)dist, tmp);
    hipLaunchKernelGGL(k_dist_sweep, dim3(grid), dim3(256), 0, s, g, periodic, solid, (const float *)tmp, dist);
  }
  NN_TRY(hipGetLastError());
  return LBM_OK;
}

extern "C" int lbm_nn_encode_geometry(int64_t n, const uint8_t *solid, const float *dist, float scale, float cap,
                                      void *x, void *stream) {
  if (!solid || !dist || !x || n < 0 || !(scale > 0.f) || !(cap > 0.f))
    return set_error(LBM_ERR_ARG, "lbm_nn_encode_geometry: args");
  hipLaunchKernelGGL(k_encode_geometry, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), n, solid,
                     dist, scale, cap, static_cast<bf16 *>(x));
  NN_TRY(hipGetLastError());
  return LBM_OK;
}

extern "C" int lbm_nn_decode_output(int64_t n, const float *pred, const uint8_t *solid, double rho0, double scale,
                                    int32_t renorm, double *rho, double *u, double *scratch, void *stream) {
  if (!pred || !solid || !rho || !u || n < 0 || (renorm && !scratch))
    return set_error(LBM_ERR_ARG, "lbm_nn_decode_output: args");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (renorm) hipLaunchKernelGGL(k_zero2, dim3(1), dim3(64), 0, s, scratch);
  hipLaunchKernelGGL(k_decode, dim3(grid_for(n)), dim3(256), 0, s, n, pred, solid, rho0, scale, rho, u,
                     renorm ? scratch : nullptr);
  if (renorm) hipLaunchKernelGGL(k_renorm, dim3(grid_for(n)), dim3(256), 0, s, n, solid, rho0, scratch, rho);
  NN_TRY(hipGetLastError());
  return LBM_OK;
}
