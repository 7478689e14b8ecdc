// Internal declarations shared by the gfx950 kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "brmppi.h"

namespace brm {

constexpr int kWChunk = 1024;     // samples per weight chunk (fixed: results never depend on
                                  // the launch shape)
constexpr int kWThreads = 256;    // threads of the reduce kernel
constexpr int kRowsPerBlock = 4;  // (step, input) rows per reduce work item: one per wave
constexpr int kPathWin = 1024;    // waypoints staged in LDS per tile
constexpr int kPathBack = 64;     // of which before the start progress
constexpr int kMaxBlock = 256;    // rollout block size bound (launch_bounds)

// Per-update descriptor read by every kernel (device memory).
struct alignas(16) SolveDesc {
  brmppi_params prm;            // 31 floats
  float inv_lambda;
  float x0[8];                  // px, py, v, a, th1, th2, delta, psi
  float t0, lambda, ds, inv_ds;
  uint32_t S, T, n_obs, flags;
  uint32_t n_path, instance, seed_lo, seed_hi;
  uint32_t S_pad, n_wchunk, n_rgroup, n_ritems;
  uint32_t x0_resident, n_normals, pad1, pad2;   // n_normals: 5 + n_obs (guided) or 3
  const float4* path;           // controller path (absolute coordinates)
  const float* u_nom_in;        // 3T nominal sequence read by the rollout
  float* u_nom_out;             // 3T warm-start slot of the controller (shift target)
  float* u_star;                // [3T][S_pad] applied inputs
  float* J;                     // [S_pad]
  float4* wpart;                // [n_wchunk] (m_c, Z_c, Z2_c, 0)
  float* rpart;                 // [n_wchunk][3T] chunk partial sums
  uint32_t* counter;            // reduce completion counter (self-resetting)
  float* u_new;                 // [3T] result
  float* stats;                 // [4] J_min, Z, ess, status
  double* plant_x;              // [8] resident plant state
  float* noise;                 // [T][n_normals][S_pad] precomputed normals (variants 1-3)
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
// with precomputed noise, 2 / 3 = two / four lanes per sample with
// precomputed noise (k_noise must run first).  All variants give bitwise
// identical results.
constexpr int kMaxVariant = 4;   // 0: G1 fused noise, 1: G1, 2: G2, 3: G4, 4: G8 (precomputed noise)
int variant_lanes(int variant);
bool variant_pre(int variant);
hipError_t launch_rollout(int bucket, int variant, const SolveDesc* descs, const Tile* tiles, uint32_t n_tiles,
                          BatchCounters* ctr, uint32_t grid, uint32_t block, hipStream_t stream);
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
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t stream);
// occupancy of a rollout variant for a bucket and block size (blocks per CU)
int rollout_blocks_per_cu(int bucket, int variant, uint32_t block);

// constraint bucket: obstacles the kernel instance can hold (0 = guidance off)
inline int bucket_for(uint32_t n_obs, uint32_t flags) {
  if (flags & BRMPPI_GUIDANCE_OFF) return 0;
  if (n_obs <= 2) return 2;
  if (n_obs <= 8) return 8;
  if (n_obs <= 16) return 16;
  return 32;
}

}  // namespace brm
