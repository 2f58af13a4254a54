/*
 * lbm_nn.h -- C ABI of the learned warm start's layer kernels (liblbm.so).
 *
 * A small 3D convolutional U-Net maps a solid mask and a force direction to
 * the steady (rho, u) of the lattice Boltzmann problem; f_eq(rho, u) then
 * initialises the solver (lbm_init), which still produces the answer.  These
 * calls are the network's building blocks; the network itself is assembled by
 * the caller.  (The method's paper has no learned component; its solver and
 * steady state are what the network imitates.)
 *
 * Conventions
 *   - Activations are BF16, one sample at a time, channels last:
 *     element (x, y, z, c) of an (nx, ny, nz) grid with row stride ld (>= the
 *     channel count, a multiple of 8) is at c + ld*(x + nx*(y + ny*z)).  Channel
 *     counts are multiples of 8; x, y and ld-strided rows are 16-byte aligned.
 *   - A layer is a gather-GEMM: for every GEMM row m (a voxel of `rows`) and
 *     output channel n,
 *         y[dst(m)][n] = act( sum_t sum_c x[src(m, t)][c] * w[n][t*cin + c] + bias[n] )
 *     src: LBM_NN_CONV3 (27 taps t = (dz+1)*9 + (dy+1)*3 + (dx+1), circular
 *     neighbour m + (dx, dy, dz)); LBM_NN_IDENT (one tap, src = m);
 *     LBM_NN_GATHER2 (8 taps t = az*4 + ay*2 + ax, src = 2m + a on a grid twice
 *     as fine).  dst: LBM_NN_IDENT, or LBM_NN_SCATTER2 (for tap t only,
 *     dst = 2m + a on a grid twice as fine: a 2x2x2 stride-2 transposed conv).
 *   - Weights w are BF16 [cout][taps*cin]; bias FP32 [cout] or NULL.
 *     Products run on BF16 MFMA (v_mfma_f32_16x16x32_bf16) with FP32
 *     accumulation.
 *   - Everything is asynchronous on the given HIP stream (NULL = default);
 *     the caller owns all buffers.  Return: LBM_OK or an LBM_ERR_* code of lbm.h.
 */
#ifndef LBM_NN_H
#define LBM_NN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_NN_IDENT 0
#define LBM_NN_CONV3 1
#define LBM_NN_GATHER2 2
#define LBM_NN_SCATTER2 3

typedef struct {
  int32_t src_mode;     /* LBM_NN_IDENT, LBM_NN_CONV3 or LBM_NN_GATHER2 */
  int32_t dst_mode;     /* LBM_NN_IDENT or LBM_NN_SCATTER2 */
  int32_t rows[3];      /* GEMM row grid (nx, ny, nz) */
  int32_t taps;         /* 27 (CONV3), 1 (IDENT), 8 (GATHER2 or SCATTER2) */
  int32_t cin, cout;    /* multiples of 8 (cout: any >= 1 for FP32 outputs) */
  const void *x;        /* BF16 input rows */
  int32_t ldx;
  const void *w;        /* BF16 [cout][taps*cin] */
  const float *bias;    /* FP32 [cout] or NULL */
  void *y;              /* output rows: BF16, or FP32 if y_fp32 */
  int32_t ldy;
  int32_t y_fp32;
  int32_t relu;         /* apply max(0, .) */
  int32_t gate_channels; /* 0, or the leading output channels that gate masks (a multiple of 8, <= cout) */
  const void *gate;     /* NULL, or BF16 rows on the output grid, stride ldg (16-byte aligned, ldg a multiple of 8) */
  int32_t ldg;
  int32_t reserved;
} lbm_nn_gemm;

/* y = act(gather-GEMM(x, w) + bias).  For LBM_NN_SCATTER2 every output voxel
 * of the fine grid is written once over the 8 taps.
 * With a gate, y[v][n] = 0 for n < gate_channels wherever gate[v][n] is not
 * greater than 0 (NaN included).  This is the derivative of a ReLU applied to
 * a backward-data pass: with gate = the layer's forward input x, itself a
 * ReLU output, the kernel writes dL/d(pre-activation) instead of dL/dx, and
 * no separate lbm_nn_relu_backward pass over the gradient is needed. */
int lbm_nn_forward(const lbm_nn_gemm *g, void *stream);

/* lbm_nn_forward with a caller workspace: on grids too small to fill the
 * device (fewer than 1024 blocks of 64 rows) with long K (at least 32 steps of
 * 32), BF16 layers without a scatter split K over S blocks per tile, each
 * writing FP32 partial sums to ws, and a second kernel adds them in a fixed
 * order (same result to rounding, identical from run to run) with bias,
 * activation and gate.  ws: device FP32, at least lbm_nn_forward_workspace(g)
 * floats, overwritten; NULL = lbm_nn_forward.  LBM_ERR_ARG if ws_floats is
 * too small. */
int lbm_nn_forward_ws(const lbm_nn_gemm *g, float *ws, int64_t ws_floats, void *stream);
/* Workspace floats lbm_nn_forward_ws uses for g (0: none); -1 for an invalid g. */
int64_t lbm_nn_forward_workspace(const lbm_nn_gemm *g);

/* Weight gradient of the same layer: dw[n][t*cin + c] += sum_m x[src(m,t)][c]
 * * dy[dst(m)][n], with g->y the BF16 gradient dy (row stride ldy) and dw an
 * FP32 [cout][taps*cin] accumulator (not cleared); g->w and g->bias unused.
 * If db is not NULL it accumulates the bias gradient, the sum of dy[v][n]
 * over every output voxel v (for SCATTER2 all 8 fine voxels of each coarse
 * one), in the same kernel (one FP32 atomic add per block and channel). */
int lbm_nn_wgrad(const lbm_nn_gemm *g, float *dw, float *db, void *stream);

/* lbm_nn_wgrad with a caller workspace: each block of the weight-gradient
 * kernel writes its partial sums there and a second kernel adds the blocks in
 * a fixed order, instead of one FP32 atomic per weight and block (same result
 * to rounding, identical from run to run, and no atomic contention).  With a
 * workspace the 3x3x3 weight gradient also takes its brick kernel on smaller
 * grids.  ws: device FP32, at least lbm_nn_wgrad_workspace(g) floats,
 * overwritten; ws may be NULL (then atomics).  LBM_ERR_ARG if ws_floats is too
 * small. */
int lbm_nn_wgrad_ws(const lbm_nn_gemm *g, float *dw, float *db, float *ws, int64_t ws_floats, void *stream);
/* Workspace floats lbm_nn_wgrad_ws needs for g; -1 for an invalid g. */
int64_t lbm_nn_wgrad_workspace(const lbm_nn_gemm *g);

/* Weights of the backward-data pass of a layer, so that lbm_nn_forward with
 * them computes dx from dy: CONV3: wt[c][t*cout + n] = w[n][(26-t)*cin + c];
 * SCATTER2 (transposed conv): wt[c][t*cout + n] = w[n][t*cin + c] (used with
 * src LBM_NN_GATHER2); IDENT: wt[c][n] = w[n][c].  BF16 in, BF16 out. */
int lbm_nn_backward_weights(int32_t mode, int32_t taps, int32_t cin, int32_t cout, const void *w, void *wt,
                            void *stream);

/* lbm_nn_backward_weights for up to LBM_NN_WT_JOBS_MAX layers in one launch
 * (mode, taps, cin, cout, w and wt as there; the jobs are read on the host and
 * the array may be reused when the call returns). */
#define LBM_NN_WT_JOBS_MAX 48
typedef struct {
  int32_t mode, taps, cin, cout;
  const void *w;
  void *wt;
} lbm_nn_wt_job;
int lbm_nn_backward_weights_batch(int32_t count, const lbm_nn_wt_job *jobs, void *stream);

/* 2x2x2 max pooling of x (fine grid 2*grid, stride ldx) into y (grid, ldy);
 * arg (uint8 per output element, c fastest over `channels`) records the
 * winning corner.  Backward: dx (fine grid, ldx) receives dy at each window's
 * winning corner and 0 elsewhere; with accumulate the values are added to dx
 * instead (for a tensor that also feeds a skip connection). */
int lbm_nn_maxpool2(const int32_t grid[3], int32_t channels, const void *x, int32_t ldx, void *y, int32_t ldy,
                    uint8_t *arg, void *stream);
int lbm_nn_maxpool2_backward(const int32_t grid[3], int32_t channels, const void *dy, int32_t ldy,
                             const uint8_t *arg, void *dx, int32_t ldx, int32_t accumulate, void *stream);

/* dy[i] = y[i] > 0 ? dy[i] : 0 over n rows of `channels` (strides ldy). */
int lbm_nn_relu_backward(int64_t n, int32_t channels, const void *y, int32_t ld_y, void *dy, int32_t ld_dy,
                         void *stream);

/* Masked mean-squared error: loss_acc[0] += sum over rows with mask == 0 of
 * sum_c (pred - target)^2 (FP32 [rows][channels]); dpred (BF16 rows of stride
 * ldd, channels written, the rest zeroed) = scale * 2 (pred - target) on those
 * rows, 0 elsewhere. */
int lbm_nn_mse(int64_t n, int32_t channels, const float *pred, const float *target, const uint8_t *mask,
               float scale, void *dpred, int32_t ldd, float *loss_acc, void *stream);

/* Adam on FP32 master weights p with moments m, v, gradient g (all n), then
 * p16 = bf16(p).  step >= 1 is the update count (bias correction). */
int lbm_nn_adam(int64_t n, float *p, float *m, float *v, const float *g, void *p16, float lr, float beta1,
                float beta2, float eps, int32_t step, void *stream);

/* Slow (Stokes) flow is linear in the body force, so the network predicts one
 * (rho - rho0, u) field per force axis and the force direction mixes them:
 * p[n][k] = sum_j dir[j] * y[n][4j + k] for k < 4 (y FP32 [nodes][12], p FP32
 * [nodes][4]).  Backward: dy[n][4j + k] = dir[j] * dp[n][k] (dp BF16 rows of
 * stride ldp; dy BF16 rows of stride ldy >= 12, entries 12.. zeroed). */
int lbm_nn_mix(int64_t n, const float *y, const float dir[3], float *p, void *stream);
int lbm_nn_mix_backward(int64_t n, const void *dp, int32_t ldp, const float dir[3], void *dy, int32_t ldy,
                        void *stream);

/* Network input: x (BF16 [nodes][8]) = (solid, gx, gy, gz on fluid nodes, 0...)
 * from a uint8 solid mask and a unit force direction. */
int lbm_nn_encode_input(int64_t n, const uint8_t *solid, const float dir[3], void *x, void *stream);

/* Distance of every node to the nearest solid node along lattice links:
 * the shortest path over D3Q19 links of length 1 (faces) or sqrt(2) (edges),
 * wrapping on periodic axes (bits as in lbm_tiles_build); 0 on solid nodes.
 * solid: device uint8 [nz][ny][nx] (shape = {nx, ny, nz}); dist, tmp: device
 * FP32 of the same size (tmp is scratch).  Each sweep is one Bellman-Ford
 * relaxation d <- min(d, d(x + c) + |c|); sweeps are run in pairs (an odd
 * count runs one more), and distances longer than about one unit per sweep
 * stay at 1e30 (also where no solid node is reachable). */
int lbm_nn_distance(const int32_t shape[3], uint32_t periodic, const uint8_t *solid, int32_t sweeps, float *dist,
                    float *tmp, void *stream);

/* Network input from the geometry: x (BF16 [nodes][8]) = (solid, s, s^2, 0, ...)
 * with s = min(dist * scale, cap) on non-solid nodes (0 on solid ones). */
int lbm_nn_encode_geometry(int64_t n, const uint8_t *solid, const float *dist, float scale, float cap, void *x,
                           void *stream);

/* Network output (FP32 [nodes][4]: scaled (rho - rho0, u)) to dense FP64
 * fields for lbm_init: rho = rho0 + s*p0, u = s*p[1..3] on fluid nodes, 0 on
 * solid ones.  If renorm, rho is shifted on fluid nodes so that its sum is
 * rho0 times the fluid count (mass of the cold start); scratch: 2 device
 * doubles. */
int lbm_nn_decode_output(int64_t n, const float *pred, const uint8_t *solid, double rho0, double scale, int32_t renorm,
                         double *rho, double *u, double *scratch, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_NN_H */
