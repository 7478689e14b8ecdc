// Internal declarations shared by the gfx950 kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "brmppi.h"

namespace brm {

// Canonical reduction structure (fixed: results never depend on the launch
// shape or on which kernel reduces): units of 32 samples weighted by their own
// minimum cost, groups of 32 units merged by log-sum-exp, then the groups.
constexpr int kUnit = 32;                    // samples per unit
constexpr int kGroupUnits = 32;              // units per group
constexpr int kWChunk = kUnit * kGroupUnits; // samples per group
constexpr int kWThreads = 256;    // threads of the reduce kernel
constexpr int kRowsPerPass = 8;   // (step, input) rows one pass of the reduce block covers: two per wave
constexpr int kMaxRowsPerItem = 256; // rows of one reduce work item (a multiple of kRowsPerPass)
constexpr int kRedBlocksPerCU = 2;   // reduce blocks a CU holds at once (its LDS and registers)
constexpr size_t kFusedLdsMax = 64 * 1024;   // dynamic LDS bound of the fused rollout
constexpr uint32_t kCtrStride = 32;          // completion counters one 128-B line apart
constexpr int kPathWin = 1024;    // waypoints staged in LDS per tile
constexpr int kPathBack = 64;     // of which before the start progress
constexpr int kMaxBlock = 256;    // rollout block size bound (launch_bounds)
constexpr int kNoisePrefetch = 2;   // steps of normals loaded ahead of their use

// Per-update descriptor read by every kernel (device memory).
struct alignas(16) SolveDesc {
  brmppi_params prm;            // 35 floats
  float inv_lambda;
  float x0[8];                  // px, py, v, a, th1, th2, delta, psi
  float t0, lambda, ds, inv_ds;
  uint32_t S, T, n_obs, flags;  // n_obs: obstacle rows (obstacles x footprint discs)
  uint32_t n_path, instance, seed_lo, seed_hi;
  uint32_t S_pad, n_wchunk, n_rgroup, n_ritems;
  uint32_t x0_resident, n_normals, fused, ustar_global;   // n_normals: 5 + n_obs (guided) or 3
  uint32_t n_units, any_e4, rows_item, any_disc;   // any_e4: some obstacle has e = 4; rows_item: rows
                                                   // of one reduce work item; any_disc: a footprint
                                                   // other than the rear axle alone
  uint32_t n_objects, pad0, pad1, pad2;          // obstacles (row r: obstacle r % n_objects, disc
                                                 // r / n_objects)
  const float4* path;           // controller path (absolute coordinates)
  const float* u_nom_in;        // 3T nominal sequence read by the rollout
  float* u_nom_out;             // 3T warm-start slot of the controller (shift target)
  float* u_star;                // [3T][S_pad] applied inputs
  float* J;                     // [S_pad]
  float4* wpart;                // [n_wchunk] group partials (m_g, Z_g, Z2_g, 0)
  float* rpart;                 // [n_wchunk][3T] group row sums
  float4* upart;                // [n_units] unit partials (m_u, Z_u, Z2_u, 0) (fused rollout)
  float* urow;                  // [n_units][3T] unit row sums (fused rollout)
  uint32_t* counter;            // instance completion counter (self-resetting)
  uint32_t* gctr;               // [n_wchunk * kCtrStride] group completion counters (fused rollout,
                                // self-resetting)
  float* u_new;                 // [3T] result
  float* stats;                 // [4] J_min, Z, ess, status
  double* plant_x;              // [8] resident plant state
  float* noise;                 // [T][n_normals][S_pad] precomputed normals (variants 1-4)
  brmppi_obstacle obs[BRMPPI_MAX_OBS];
};

struct Tile { uint32_t inst, s0; };
struct Item { uint32_t inst, idx; };

// Work counters of the persistent kernels of one stream (device memory; the
// last block of each kernel resets them to zero).
struct alignas(16) BatchCounters {
  uint32_t tile_next, tile_done, r_next, r_done;
};

// Launchers (kernels.hip).  All enqueue on `stream` and return hipError_t.
// Rollout variant: 0 = one lane per sample with in-kernel noise, 1 = one lane
// with precomputed noise, 2 / 3 / 4 = two / four / eight lanes per sample
// with precomputed noise (k_noise must run first).  All variants give bitwise
// identical results.
constexpr int kMaxVariant = 4;   // 0: G1 fused noise, 1: G1, 2: G2, 3: G4, 4: G8 (precomputed noise)
int variant_lanes(int variant);
bool variant_pre(int variant);
// lds_bytes > 0: the single instance's tiles reduce themselves (fused epilogue;
// descs->fused must be set and the tile size a multiple of kUnit)
hipError_t launch_rollout(int bucket, int variant, const SolveDesc* descs, const Tile* tiles, uint32_t n_tiles,
                          BatchCounters* ctr, uint32_t grid, uint32_t block, size_t lds_bytes, hipStream_t stream);
// dynamic LDS of the fused epilogue for a tile of `per_tile` samples: the
// tile's applied inputs [3T][per_tile + 1] (later reused for the n_groups
// merge scales), costs, weights, unit minima and scales, unit partials
__host__ __device__ inline size_t fused_lds_region(uint32_t per_tile, uint32_t T, uint32_t n_groups) {
  const size_t a = (size_t)3 * T * (per_tile + 1);
  return ((a > n_groups ? a : n_groups) + 3) / 4 * 4;
}
// a tile can reduce itself only when it holds whole units and the tiles cover
// each group of kWChunk samples exactly (no tile straddles two groups, so a
// group has ceil(units / units per tile) tiles)
__host__ __device__ inline bool fused_tile_ok(uint32_t per_tile) {
  return per_tile > 0 && per_tile % kUnit == 0 && kWChunk % per_tile == 0;
}
__host__ __device__ inline size_t fused_lds_bytes(uint32_t per_tile, uint32_t T, uint32_t n_groups) {
  return sizeof(float) * (fused_lds_region(per_tile, T, n_groups) + 2 * (size_t)per_tile + 2 * kGroupUnits) +
         16 * kGroupUnits;
}
// normals of `count` instances whose descriptors start at `first`, `stride`
// bytes apart (all with the same S, T and normals per step)
hipError_t launch_noise(const SolveDesc* first, size_t stride, uint32_t count, uint32_t S, uint32_t T,
                        uint32_t n_normals, hipStream_t stream);
hipError_t launch_reduce(const SolveDesc* descs, const Item* items, uint32_t n_items,
                         BatchCounters* ctr, uint32_t grid, hipStream_t stream);
hipError_t launch_philox_dump(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t n, uint32_t* out,
                              hipStream_t stream);
hipError_t launch_normals_dump(uint32_t seed_lo, uint32_t seed_hi, uint32_t instance, const uint32_t* s_tau,
                               uint32_t n, uint32_t K, float* out, hipStream_t stream);
hipError_t launch_box_muller_dump(const uint32_t* r, uint32_t n, float* out, hipStream_t stream);
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t stream);
// occupancy of a rollout variant for a bucket and block size (blocks per CU)
int rollout_blocks_per_cu(int bucket, int variant, uint32_t block);

// footprint discs of a parameter set, and whether it is other than the rear
// axle alone (the point eq. (16) uses)
inline uint32_t n_discs(const brmppi_params& P) { return P.n_disc_tractor + P.n_disc_trailer; }
inline bool footprint_is_rear_axle(const brmppi_params& P) {
  return P.n_disc_tractor == 1 && P.n_disc_trailer == 0 && P.disc_tractor[0] == 0.0f;
}
// (A, B) of disc k in row order: centre p + A e1 - B f2 (tractor discs ahead of
// the rear axle, then trailer discs behind the hitch, lh behind the rear axle)
__host__ __device__ inline void disc_ab(const brmppi_params& P, uint32_t k, float& A, float& B) {
  if (k < P.n_disc_tractor) {
    A = P.disc_tractor[k];
    B = 0.0f;
  } else {
    A = -P.lh;
    B = P.disc_trailer[k - P.n_disc_tractor];
  }
}

// constraint bucket: obstacle rows the kernel instance can hold (0 = guidance off)
inline int bucket_for(uint32_t n_obs, uint32_t flags) {
  if (flags & BRMPPI_GUIDANCE_OFF) return 0;
  if (n_obs <= 2) return 2;
  if (n_obs <= 8) return 8;
  if (n_obs <= 16) return 16;
  return 32;
}

}  // namespace brm
