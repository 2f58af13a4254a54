// Host-callable launchers of the liblbm kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace lbm {

struct TileArgs;
struct SampleRec;
struct CollideCoef;
struct NbRec;

// Compile-time variant of the kernels: lattice, tile shape, storage form and
// waves per workgroup of the step kernel.
struct Variant {
  int q;           // 9 or 19
  int ax, ay, az;  // tile edges
  int storage;     // LBM_F64 / LBM_F32_OFFSET / LBM_F16_OFFSET
  int wpb;         // waves per workgroup (D2Q9 16x16: 4 = one tile)
  int model;       // LBM_MODEL_*
  int collision;   // LBM_COLLISION_*
};

bool variant_supported(const Variant &v);
int storage_bytes(int storage);

// phase: kPhase* of device.h
hipError_t launch_step(const Variant &v, int phase, const void *src, void *dst, const TileArgs &a, double omega,
                       hipStream_t s);
// D3Q19 4x4x4 step with scalar-mask addressing (step19.hip); needs PDF entry
// indices below 2^32.
bool step19_supported(const Variant &v);
// nrec: n_ftiles + 1 records (the last one all-solid); nrow: 20 per tile, the
// byte offsets into nrec of the 18 neighbour slots of the D3Q19 gather in
// kernel order (+2 padding); rbase: kRegionBases per tile, the base entry
// index of every lane region (device.h).
// mode 0: wavefront w -> tile w; 1: -> list[w] for w < *count; 2: persistent
// grid of blocks_persistent workgroups striding over list[0 .. *count).
// shuffle: the two-copy step in its shuffle form (own values loaded
// coalesced, in-tile sources taken from other lanes; step19.hip).
hipError_t launch_step19(const Variant &v, int phase, bool shuffle, const void *src, void *dst, const TileArgs &a,
                         const NbRec *nrec, const uint32_t *nrow, const uint32_t *rbase, const CollideCoef *coef,
                         bool nontemporal, const int32_t *list, const int32_t *count, int mode,
                         int64_t blocks_persistent, hipStream_t s);
// Workgroups of the persistent step resident at once (for both single-copy
// phases when single_copy).
hipError_t step19_persistent_blocks(const Variant &v, bool single_copy, bool shuffle, int64_t *blocks);
hipError_t launch_init(const Variant &v, void *dst, const TileArgs &a, const double *rho, const double *u,
                       hipStream_t s);
hipError_t launch_moments(const Variant &v, const void *src, const TileArgs &a, double *rho, double *u,
                          hipStream_t s);
hipError_t launch_export(const Variant &v, const void *src, const TileArgs &a, double *dense, hipStream_t s);
hipError_t launch_import(const Variant &v, void *dst, const TileArgs &a, const double *dense, hipStream_t s);
// Moving wall: add the wall's term to the bounce-back entries that the lid
// nodes of the listed tiles pull next step (slot opp(i) of the two-copy
// source when own_slot == 0, slot i of the single copy when 1).
hipError_t launch_lid_fixup(const Variant &v, void *buf, const TileArgs &a, const int32_t *tiles, int64_t n_tiles,
                            int own_slot, hipStream_t s);
// per-wave partial sums: 4 per wave (mass, rho u) ...
hipError_t launch_reduce_partial(const Variant &v, const void *src, const TileArgs &a, double *part,
                                 hipStream_t s);
// ... and 2 per wave (|u - u_ref|^2, |u|^2), updating u_ref ([3][n_fluid])
hipError_t launch_residual_partial(const Variant &v, const void *src, const TileArgs &a, double *uref,
                                   double *part, int accumulate, hipStream_t s);
// fixed-order sum of per-wave partials over each sample's waves; chunk is
// scratch of reduce_chunks() * ncomp doubles per sample
int reduce_chunks();
hipError_t launch_reduce_final(const double *part, int ncomp, const SampleRec *samples, int n_samples,
                               int words, double *chunk, double *out, hipStream_t s);
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s);

}  // namespace lbm
