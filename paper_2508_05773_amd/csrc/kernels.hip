// gfx950 kernels of one BR-MPPI control update (arXiv 2508.05773).
//
//   k_rollout : counter-based noise + S rollouts of the tractor-trailer model,
//               each step projected onto the barrier-rate equalities (eq. (9))
//               with the soft-bound closed form (eqs. (11)-(12)), contouring
//               cost (eqs. (13)-(15)) accumulated; writes the applied inputs
//               [3T][S] and the cost of every sample.
//   k_weights : per 1024-sample chunk, min cost and sum of
//               exp(-(J - m_chunk)/lambda) (Sec. III-B weights).
//   k_reduce  : chunk partials of sum_s gamma_s u*_s for every (step, input)
//               row, then the last block of the instance merges the chunks
//               (log-sum-exp rescaling), writes the new nominal sequence
//               (eq. (5)) and the receding-horizon shift (Sec. III-B).
//   k_plant   : closed-loop helper: advance a resident FP64 plant by the first
//               averaged input (eq. (6)).
//
// One lane owns one sample; its state, barrier rates and row terms stay in
// registers.  Obstacles (with their shape matrices) and a window of the path
// are staged in LDS per tile.  Positions are carried relative to the start
// position and progress relative to the start progress so that FP32 keeps
// sub-micrometre resolution far from the origin.
#include <math.h>

#include "brmppi_internal.h"

namespace brm {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64 products,
// Weyl-sequence key schedule.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// (r >> 9 + 1/2) / 2^23: exact in FP32
__device__ __forceinline__ float unif23(uint32_t r) {
  return (float)(r >> 9) * 0x1p-23f + 0x1p-24f;
}

// Box-Muller on the pairs (u0, u1) and (u2, u3)
__device__ __forceinline__ void box_muller4(const uint32_t r[4], float* n) {
  const float u0 = unif23(r[0]), u1 = unif23(r[1]), u2 = unif23(r[2]), u3 = unif23(r[3]);
  const float rad0 = sqrtf(-2.0f * logf(u0));
  const float rad1 = sqrtf(-2.0f * logf(u2));
  float s1, c1, s3, c3;
  sincospif(2.0f * u1, &s1, &c1);
  sincospif(2.0f * u3, &s3, &c3);
  n[0] = rad0 * c1;
  n[1] = rad0 * s1;
  n[2] = rad1 * c3;
  n[3] = rad1 * s3;
}

constexpr float kTwoPi = 6.283185307179586f;
constexpr float kInvTwoPi = 0.15915494309189535f;

__device__ __forceinline__ float wrap_angle(float x) { return x - kTwoPi * rintf(x * kInvTwoPi); }

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Obstacle staged in LDS: centre relative to the tile origin, velocity, shape
// matrix Q = R' diag((mx+r)^-2, (my+r)^-2) R of eq. (16) with e = 2.
struct ObsL {
  float cx, cy, vx, vy, q11, q12, q22, pad;
};

struct RefPoint {
  float x, y, th1, th2;
};

// Reference zeta(psi): linear interpolation between waypoints, headings by the
// wrapped difference, clamped to the ends.  f = phi0 + psi_rel/ds is the
// fractional waypoint index relative to k0.
__device__ __forceinline__ RefPoint reference(float f, int k0, int n_path, const float4* __restrict__ spath,
                                              int w0, int nw, const float4* __restrict__ gpath, float ox,
                                              float oy) {
  float fi = floorf(f);
  fi = fminf(fmaxf(fi, -1.0e7f), 1.0e7f);  // NaN -> -1e7 -> clamped to the start
  float t = f - fi;
  int gi = k0 + (int)fi;
  if (gi < 0) {
    gi = 0;
    t = 0.0f;
  } else if (gi > n_path - 2) {
    gi = n_path - 2;
    t = 1.0f;
  }
  if (!(t >= 0.0f)) t = 0.0f;
  float4 A, B;
  const int li = gi - w0;
  if (li >= 0 && li + 1 < nw) {
    A = spath[li];
    B = spath[li + 1];
  } else {
    A = gpath[gi];
    B = gpath[gi + 1];
    A.x -= ox;
    A.y -= oy;
    B.x -= ox;
    B.y -= oy;
  }
  RefPoint r;
  r.x = A.x + t * (B.x - A.x);
  r.y = A.y + t * (B.y - A.y);
  r.th1 = A.z + t * wrap_angle(B.z - A.z);
  r.th2 = A.w + t * wrap_angle(B.w - A.w);
  return r;
}

// Tracking part of eq. (13): contour (14), lag (15) and heading errors.
__device__ __forceinline__ float tracking_cost(const brmppi_params& P, const RefPoint& rf, float px, float py,
                                               float th1, float th2) {
  float sr, cr;
  sincosf(rf.th1, &sr, &cr);
  const float ex = px - rf.x, ey = py - rf.y;
  const float ec = sr * ex - cr * ey;
  const float el = -cr * ex - sr * ey;
  const float e1 = wrap_angle(th1 - rf.th1);
  const float e2 = wrap_angle(th2 - rf.th2);
  return P.Qc * ec * ec + P.Ql * el * el + P.Qth1 * e1 * e1 + P.Qth2 * e2 * e2;
}

// ---------------------------------------------------------------------------
// Rollout
// ---------------------------------------------------------------------------
template <int NOB, bool GUIDED>
__device__ __forceinline__ void rollout_sample(const SolveDesc& d, uint32_t s, const float* x0,
                                               const ObsL* __restrict__ sobs, const float4* __restrict__ spath,
                                               int w0, int nw, int k0, float phi0) {
  constexpr int NR = NOB + 2;                       // rows: hitch+, hitch-, obstacles
  constexpr int NBMAX = GUIDED ? (5 + NOB + 3) / 4 : 1;
  const brmppi_params& P = d.prm;
  const float Ts = P.Ts, Ts2 = P.Ts * P.Ts;
  const float inv_l1 = 1.0f / P.l1, inv_l2 = 1.0f / P.l2, ch = P.lh / P.l1;
  const int n_obs = (int)d.n_obs;
  const bool hitch = !(d.flags & BRMPPI_HITCH_OFF);
  // an unguided instance may share a guided launch: the flag is honoured here
  const bool guided = GUIDED && !(d.flags & BRMPPI_GUIDANCE_OFF);
  const int nb = guided ? (5 + n_obs + 3) / 4 : 1;
  const float ox = x0[0], oy = x0[1];
  const float4* __restrict__ gpath = d.path;
  const int n_path = (int)d.n_path;

  // soft-bound projection constants, eq. (11): M = W + rho I,
  // p = W z_des + rho/2 (lo + hi)
  const float Mj = P.W_j + P.rho, Mw = P.W_w + P.rho, Ma = P.W_a + P.rho;
  const float inv_Ma = 1.0f / Ma;
  const float pj0 = 0.5f * P.rho * (P.j_lo + P.j_hi);
  const float pw0 = 0.5f * P.rho * (P.w_lo + P.w_hi);
  const float amid = 0.5f * (P.alpha_lo + P.alpha_hi);

  float px = 0.0f, py = 0.0f, v = x0[2], a = x0[3], th1 = x0[4], th2 = x0[5], dl = x0[6], psi = 0.0f;
  float alpha[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) alpha[i] = P.alpha0;
  double J = 0.0;
  const uint32_t S_pad = d.S_pad;
  float* __restrict__ ustar = d.u_star;
  const float* __restrict__ unom = d.u_nom_in;

  for (uint32_t tau = 0; tau < d.T; ++tau) {
    // --- noise (Philox counter (s, tau, block, instance), key = seed) ---
    float eps[4 * NBMAX];
#pragma unroll
    for (int b = 0; b < NBMAX; ++b) {
      if (b < nb) {
        uint32_t r[4];
        philox4x32_10(s, tau, (uint32_t)b, d.instance, d.seed_lo, d.seed_hi, r);
        box_muller4(r, &eps[4 * b]);
      }
    }
    float uj = unom[3 * tau + 0] + P.sigma_j * eps[0];
    float uw = unom[3 * tau + 1] + P.sigma_w * eps[1];
    const float unu = unom[3 * tau + 2] + P.sigma_nu * eps[2];

    float s1, c1, sp, cp;
    sincosf(th1, &s1, &c1);
    sincosf(th1 - th2, &sp, &cp);
    const float tn = tanf(dl);
    const float kd = tn * inv_l1;     // th1_dot = v kd
    const float vkd = v * kd;
    const float Aw2 = sp - ch * cp * tn;

    if (GUIDED && guided) {
      const float sec2 = 1.0f + tn * tn;
      const float t = d.t0 + (float)tau * Ts;
      // 2x2 normal equations of the eliminated projection, in FP64:
      // (M_u + sum c_i g_i g_i') u = p_u + sum c_i g_i r_i
      double N00 = Mj, N01 = 0.0, N11 = Mw;
      double y0 = (double)(P.W_j * uj + pj0), y1 = (double)(P.W_w * uw + pw0);
      float rLf[NR], rg0[NR], rg1[NR], rih[NR];

      auto accumulate = [&](int i, float hhat, float Lf, float g0, float g1, float atil) {
        const float ah = fabsf(hhat);
        const float hh = (ah < P.h_eps) ? (hhat < 0.0f ? -P.h_eps : P.h_eps) : hhat;
        const float b = -Lf - alpha[i] * hh;
        const float abar = (P.W_a * atil + P.rho * (amid - alpha[i])) * inv_Ma;
        const float rr = b - hh * abar;
        const float ih = rcp(hh);
        const float c = Ma * ih * ih;
        const double cg0 = (double)c * (double)g0, cg1 = (double)c * (double)g1;
        N00 = fma(cg0, (double)g0, N00);
        N01 = fma(cg0, (double)g1, N01);
        N11 = fma(cg1, (double)g1, N11);
        y0 = fma(cg0, (double)rr, y0);
        y1 = fma(cg1, (double)rr, y1);
        rLf[i] = Lf;
        rg0[i] = g0;
        rg1[i] = g1;
        rih[i] = ih;
      };

      // hitch rows, eq. (18) split into h_s = dth_max - kappa v + s (th1 - th2),
      // first-order expansion hhat = h + Ts hd
      if (hitch) {
        const float D = v * inv_l2 * Aw2 - vkd;                 // th2_dot - th1_dot
        const float D_v = inv_l2 * Aw2 - kd;
        const float D_phi = v * inv_l2 * (cp + ch * sp * tn);
        const float D_dl = -v * sec2 * (inv_l2 * ch * cp + inv_l1);
        const float phi = th1 - th2;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const float sg = k == 0 ? 1.0f : -1.0f;
          const float h = P.dtheta_max - P.kappa * v + sg * phi;
          const float hd = -P.kappa * a - sg * D;
          const float hv = -P.kappa - sg * Ts * D_v;
          const float Lf = Ts * (hv * a - sg * (1.0f - Ts * D_phi) * D);
          accumulate(k, h + Ts * hd, Lf, -P.kappa * Ts2, -sg * Ts2 * D_dl, P.sigma_a * eps[3 + k]);
        }
      }
      // obstacle rows, eqs. (16)-(17): with q = d + Ts d_dot,
      // hhat = q'Qq - 1 + Ts^2 d'Q d_ddot
#pragma unroll
      for (int o = 0; o < NOB; ++o) {
        if (o < n_obs) {
          const ObsL ob = sobs[o];
          const float dx = px - (ob.cx + ob.vx * t), dy = py - (ob.cy + ob.vy * t);
          const float ddx = v * c1 - ob.vx, ddy = v * s1 - ob.vy;
          const float v2kd = v * vkd;
          const float dddx = a * c1 - v2kd * s1, dddy = a * s1 + v2kd * c1;
          const float qx = dx + Ts * ddx, qy = dy + Ts * ddy;
          const float Qqx = ob.q11 * qx + ob.q12 * qy, Qqy = ob.q12 * qx + ob.q22 * qy;
          const float Qdx = ob.q11 * dx + ob.q12 * dy, Qdy = ob.q12 * dx + ob.q22 * dy;
          const float hhat = qx * Qqx + qy * Qqy - 1.0f + Ts2 * (Qdx * dddx + Qdy * dddy);
          const float dQe1 = Qdx * c1 + Qdy * s1, dQe2 = Qdy * c1 - Qdx * s1;
          const float qQe1 = Qqx * c1 + Qqy * s1, qQe2 = Qqy * c1 - Qqx * s1;
          // gradient of hhat: position, speed, heading, time
          const float gpx = 2.0f * Qqx + Ts2 * (ob.q11 * dddx + ob.q12 * dddy);
          const float gpy = 2.0f * Qqy + Ts2 * (ob.q12 * dddx + ob.q22 * dddy);
          const float h_v = 2.0f * Ts * qQe1 + 2.0f * Ts2 * vkd * dQe2;
          const float h_th = 2.0f * Ts * v * qQe2 + Ts2 * (a * dQe2 - v2kd * dQe1);
          const float h_t = -(gpx * ob.vx + gpy * ob.vy);
          const float Lf = Ts * (v * (gpx * c1 + gpy * s1) + h_v * a + h_th * vkd + h_t);
          const float g0 = Ts * Ts2 * dQe1;                          // Ts d hhat/da
          const float g1 = Ts * Ts2 * v * v * sec2 * inv_l1 * dQe2;   // Ts d hhat/d delta
          accumulate(2 + o, hhat, Lf, g0, g1, P.sigma_a * eps[5 + o]);
        }
      }
      const double det = N00 * N11 - N01 * N01;
      const double idet = 1.0 / det;
      const double u0 = (N11 * y0 - N01 * y1) * idet;
      const double u1 = (N00 * y1 - N01 * y0) * idet;
      uj = (float)u0;
      uw = (float)u1;
      // next barrier rates: alpha + u*alpha = -(Lf + g u*)/hh (eq. (9) holds exactly)
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const bool on = (i < 2) ? hitch : (i - 2 < n_obs);
        if (on) alpha[i] = -(rLf[i] + rg0[i] * uj + rg1[i] * uw) * rih[i];
      }
    }

    // --- stage cost r(x_tau, u*_tau, psi_tau), eq. (13) ---
    const RefPoint rf = reference(phi0 + psi * d.inv_ds, k0, n_path, spath, w0, nw, gpath, ox, oy);
    const float prog = P.nu_bar - unu;
    const float rc = tracking_cost(P, rf, px, py, th1, th2) + P.R_j * uj * uj + P.R_w * uw * uw +
                     P.mu * prog * prog;
    J += (double)rc;

    // --- applied inputs [3T][S_pad] ---
    ustar[(size_t)(3 * tau + 0) * S_pad + s] = uj;
    ustar[(size_t)(3 * tau + 1) * S_pad + s] = uw;
    ustar[(size_t)(3 * tau + 2) * S_pad + s] = unu;

    // --- explicit Euler, eq. (6), plus psi_dot = nu ---
    const float npx = px + Ts * v * c1;
    const float npy = py + Ts * v * s1;
    const float nv = v + Ts * a;
    const float na = a + Ts * uj;
    const float nth1 = th1 + Ts * vkd;
    const float nth2 = th2 + Ts * v * inv_l2 * Aw2;
    const float ndl = dl + Ts * uw;
    psi += Ts * unu;
    px = npx;
    py = npy;
    v = nv;
    a = na;
    th1 = nth1;
    th2 = nth2;
    dl = ndl;
  }
  const RefPoint rf = reference(phi0 + psi * d.inv_ds, k0, n_path, spath, w0, nw, gpath, ox, oy);
  J += (double)tracking_cost(P, rf, px, py, th1, th2);
  float Jf = (float)J;
  if (!isfinite(Jf)) Jf = INFINITY;
  d.J[s] = Jf;
}

template <int NOB, bool GUIDED>
__global__ __launch_bounds__(kMaxBlock) void k_rollout(const SolveDesc* __restrict__ descs,
                                                       const Tile* __restrict__ tiles, uint32_t n_tiles,
                                                       BatchCounters* __restrict__ ctr) {
  __shared__ float4 s_path[kPathWin];
  __shared__ ObsL s_obs[BRMPPI_MAX_OBS > 0 ? BRMPPI_MAX_OBS : 1];
  __shared__ uint32_t s_tile;
  for (uint32_t it = 0;; ++it) {
    uint32_t tix;
    if (ctr) {
      if (threadIdx.x == 0) s_tile = atomicAdd(&ctr->tile_next, 1u);
      __syncthreads();
      tix = s_tile;
    } else {
      if (it > 0) break;
      tix = blockIdx.x;
    }
    tix = __builtin_amdgcn_readfirstlane(tix);
    if (tix >= n_tiles) break;
    Tile tl;
    if (tiles) {
      tl = tiles[tix];
    } else {
      tl.inst = 0;
      tl.s0 = tix * blockDim.x;
    }
    const SolveDesc& d = descs[__builtin_amdgcn_readfirstlane(tl.inst)];

    float x0[8];
    if (d.x0_resident) {
#pragma unroll
      for (int k = 0; k < 8; ++k) x0[k] = (float)d.plant_x[k];
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) x0[k] = d.x0[k];
    }
    const float ox = x0[0], oy = x0[1];
    // progress origin: f0 = psi0/ds = k0 + phi0
    const double f0 = (double)x0[7] / (double)d.ds;
    double fk = floor(f0);
    fk = fmin(fmax(fk, -1.0e9), 1.0e9);
    const int k0 = (int)fk;
    const float phi0 = (float)(f0 - fk);
    const int n_path = (int)d.n_path;
    int w0 = k0 - kPathBack;
    if (w0 < 0) w0 = 0;
    if (w0 > n_path - 2) w0 = n_path - 2;
    int nw = n_path - w0;
    if (nw > kPathWin) nw = kPathWin;

    // stage obstacles (shape matrices) and the path window
    if (threadIdx.x < d.n_obs) {
      const brmppi_obstacle o = d.obs[threadIdx.x];
      const float ax = o.mx + d.prm.r_disc, ay = o.my + d.prm.r_disc;
      const float iax = 1.0f / (ax * ax), iay = 1.0f / (ay * ay);
      float so, co;
      sincosf(o.heading, &so, &co);
      ObsL L;
      L.cx = o.cx - ox;
      L.cy = o.cy - oy;
      L.vx = o.vx;
      L.vy = o.vy;
      L.q11 = co * co * iax + so * so * iay;
      L.q12 = co * so * (iax - iay);
      L.q22 = so * so * iax + co * co * iay;
      L.pad = 0.0f;
      s_obs[threadIdx.x] = L;
    }
    for (int j = threadIdx.x; j < nw; j += blockDim.x) {
      float4 w = d.path[w0 + j];
      w.x -= ox;
      w.y -= oy;
      s_path[j] = w;
    }
    __syncthreads();

    const uint32_t s = tl.s0 + threadIdx.x;
    if (s < d.S) rollout_sample<NOB, GUIDED>(d, s, x0, s_obs, s_path, w0, nw, k0, phi0);
    __syncthreads();
  }
  if (ctr && threadIdx.x == 0) {
    __threadfence();
    const uint32_t done = atomicAdd(&ctr->tile_done, 1u);
    if (done == gridDim.x - 1) {
      atomicExch(&ctr->tile_next, 0u);
      atomicExch(&ctr->tile_done, 0u);
    }
  }
}

// ---------------------------------------------------------------------------
// Block reductions (deterministic: fixed butterfly, fixed wave order)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fminf(v, __shfl_xor(v, m, 64));
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// grab the next work item (persistent) or take blockIdx.x (direct launch)
__device__ __forceinline__ bool next_item(uint32_t it, uint32_t n_items, uint32_t* ctr_next, uint32_t* s_slot,
                                          uint32_t& ix) {
  if (ctr_next) {
    if (threadIdx.x == 0) *s_slot = atomicAdd(ctr_next, 1u);
    __syncthreads();
    ix = *s_slot;
  } else {
    if (it > 0) return false;
    ix = blockIdx.x;
  }
  ix = __builtin_amdgcn_readfirstlane(ix);
  return ix < n_items;
}

__device__ __forceinline__ void finish_persistent(uint32_t* next, uint32_t* done) {
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t k = atomicAdd(done, 1u);
    if (k == gridDim.x - 1) {
      atomicExch(next, 0u);
      atomicExch(done, 0u);
    }
  }
}

// ---------------------------------------------------------------------------
// Weights: per chunk m_c = min J, gamma = exp(-(J - m_c)/lambda), Z_c, Z2_c
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWThreads) void k_weights(const SolveDesc* __restrict__ descs,
                                                      const Item* __restrict__ items, uint32_t n_items,
                                                      BatchCounters* __restrict__ ctr) {
  __shared__ float s_red[3][kWThreads / 64];
  __shared__ uint32_t s_slot;
  constexpr int PER = kWChunk / kWThreads;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (uint32_t it = 0;; ++it) {
    uint32_t ix;
    if (!next_item(it, n_items, ctr ? &ctr->w_next : nullptr, &s_slot, ix)) break;
    Item item;
    if (items) item = items[ix];
    else {
      item.inst = 0;
      item.idx = ix;
    }
    const SolveDesc& d = descs[__builtin_amdgcn_readfirstlane(item.inst)];
    const uint32_t base = item.idx * kWChunk;
    float Jv[PER];
    float m = INFINITY;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const uint32_t s = base + threadIdx.x + j * kWThreads;
      float x = (s < d.S) ? d.J[s] : INFINITY;
      if (!(x < INFINITY)) x = INFINITY;  // NaN -> +inf (weight 0)
      Jv[j] = x;
      m = fminf(m, x);
    }
    m = wave_min(m);
    if (lane == 0) s_red[0][wid] = m;
    __syncthreads();
    m = s_red[0][0];
#pragma unroll
    for (int w = 1; w < kWThreads / 64; ++w) m = fminf(m, s_red[0][w]);
    float z = 0.0f, z2 = 0.0f;
    const bool any = m < INFINITY;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const uint32_t s = base + threadIdx.x + j * kWThreads;
      const float g = (any && Jv[j] < INFINITY) ? expf(-(Jv[j] - m) * d.inv_lambda) : 0.0f;
      if (s < d.S) d.gam[s] = g;
      z += g;
      z2 += g * g;
    }
    z = wave_sum(z);
    z2 = wave_sum(z2);
    __syncthreads();
    if (lane == 0) {
      s_red[1][wid] = z;
      s_red[2][wid] = z2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      float Z = 0.0f, Z2 = 0.0f;
#pragma unroll
      for (int w = 0; w < kWThreads / 64; ++w) {
        Z += s_red[1][w];
        Z2 += s_red[2][w];
      }
      d.wpart[item.idx] = make_float4(m, Z, Z2, 0.0f);
    }
    __syncthreads();
  }
  if (ctr) finish_persistent(&ctr->w_next, &ctr->w_done);
}

// ---------------------------------------------------------------------------
// Reduce: rows of the applied-input tensor weighted by gamma, per chunk; the
// last block of an instance merges chunks and writes the update + shift.
// ---------------------------------------------------------------------------
__device__ void finalize_instance(const SolveDesc& d, float* s_scale, float* s_misc) {
  const uint32_t nW = d.n_wchunk;
  const uint32_t R = 3 * d.T;
  // merge chunk partials (fixed order)
  if (threadIdx.x == 0) {
    float m = INFINITY;
    for (uint32_t c = 0; c < nW; ++c) m = fminf(m, d.wpart[c].x);
    float Z = 0.0f, Z2 = 0.0f;
    if (m < INFINITY) {
      for (uint32_t c = 0; c < nW; ++c) {
        const float4 w = d.wpart[c];
        const float sc = (w.x < INFINITY) ? expf(-(w.x - m) * d.inv_lambda) : 0.0f;
        s_scale[c] = sc;
        Z += sc * w.y;
        Z2 += sc * sc * w.z;
      }
    }
    s_misc[0] = m;
    s_misc[1] = Z;
    s_misc[2] = Z2;
  }
  __syncthreads();
  const float m = s_misc[0], Z = s_misc[1], Z2 = s_misc[2];
  const bool ok = (m < INFINITY) && (Z > 0.0f);
  if (ok) {
    const float iZ = 1.0f / Z;
    for (uint32_t r = threadIdx.x; r < R; r += blockDim.x) {
      float acc = 0.0f;
      for (uint32_t c = 0; c < nW; ++c) acc += s_scale[c] * d.rpart[(size_t)c * R + r];
      const float U = acc * iZ;
      d.u_new[r] = U;
      // receding-horizon shift: U_nom <- [U[1:], U[T-1]]
      if (r >= 3) d.u_nom_out[r - 3] = U;
      if (r + 3 >= R) d.u_nom_out[r] = U;
    }
  } else {
    // every cost non-finite: return the nominal sequence, keep the warm start
    for (uint32_t r = threadIdx.x; r < R; r += blockDim.x) d.u_new[r] = d.u_nom_in[r];
  }
  if (threadIdx.x == 0) {
    d.stats[0] = m;
    d.stats[1] = Z;
    d.stats[2] = ok ? Z * Z / Z2 : 0.0f;
    d.stats[3] = ok ? (float)BRMPPI_OK : (float)BRMPPI_ENONFINITE;
  }
}

constexpr uint32_t kMaxWChunks = BRMPPI_MAX_S / kWChunk;

__global__ __launch_bounds__(kWThreads) void k_reduce(const SolveDesc* __restrict__ descs,
                                                     const Item* __restrict__ items, uint32_t n_items,
                                                     BatchCounters* __restrict__ ctr) {
  __shared__ float s_part[kRowsPerBlock][kWThreads / 64];
  __shared__ float s_scale[kMaxWChunks];
  __shared__ float s_misc[4];
  __shared__ uint32_t s_slot, s_last;
  constexpr int PER = kWChunk / kWThreads;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (uint32_t it = 0;; ++it) {
    uint32_t ix;
    if (!next_item(it, n_items, ctr ? &ctr->r_next : nullptr, &s_slot, ix)) break;
    Item item;
    if (items) item = items[ix];
    else {
      item.inst = 0;
      item.idx = ix;
    }
    const SolveDesc& d = descs[__builtin_amdgcn_readfirstlane(item.inst)];
    const uint32_t chunk = item.idx / d.n_rgroup, rg = item.idx % d.n_rgroup;
    const uint32_t base = chunk * kWChunk;
    const uint32_t R = 3 * d.T;
    float g[PER];
    uint32_t sj[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      sj[j] = base + threadIdx.x + j * kWThreads;
      g[j] = (sj[j] < d.S) ? d.gam[sj[j]] : 0.0f;
    }
    const uint32_t r0 = rg * kRowsPerBlock;
#pragma unroll
    for (int q = 0; q < kRowsPerBlock; ++q) {
      const uint32_t r = r0 + q;
      float acc = 0.0f;
      if (r < R) {
        const float* __restrict__ row = d.u_star + (size_t)r * d.S_pad;
#pragma unroll
        for (int j = 0; j < PER; ++j)
          if (sj[j] < d.S) acc += g[j] * row[sj[j]];
      }
      acc = wave_sum(acc);
      if (lane == 0) s_part[q][wid] = acc;
    }
    __syncthreads();
    if (threadIdx.x < kRowsPerBlock) {
      const uint32_t r = r0 + threadIdx.x;
      if (r < R) {
        float v = 0.0f;
#pragma unroll
        for (int w = 0; w < kWThreads / 64; ++w) v += s_part[threadIdx.x][w];
        d.rpart[(size_t)chunk * R + r] = v;
      }
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
      const uint32_t k = atomicAdd(d.counter, 1u);
      s_last = (k == d.n_ritems - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (s_last) {
      __threadfence();
      finalize_instance(d, s_scale, s_misc);
      if (threadIdx.x == 0) atomicExch(d.counter, 0u);
    }
    __syncthreads();
  }
  if (ctr) finish_persistent(&ctr->r_next, &ctr->r_done);
}

// ---------------------------------------------------------------------------
// Closed-loop plant: x <- Euler(x, clamp(U_new[0])) in FP64 (eq. (6))
// ---------------------------------------------------------------------------
__device__ void plant_step(const SolveDesc& d) {
  const brmppi_params& P = d.prm;
  double x[8];
  for (int k = 0; k < 8; ++k) x[k] = d.plant_x[k];
  double j = d.u_new[0], w = d.u_new[1], nu = d.u_new[2];
  j = fmin(fmax(j, (double)P.j_lo), (double)P.j_hi);
  w = fmin(fmax(w, (double)P.w_lo), (double)P.w_hi);
  const double Ts = P.Ts, l1 = P.l1, l2 = P.l2, lh = P.lh;
  const double v = x[2], a = x[3], t1 = x[4], t2 = x[5], dl = x[6];
  double xn[8];
  xn[0] = x[0] + Ts * v * cos(t1);
  xn[1] = x[1] + Ts * v * sin(t1);
  xn[2] = v + Ts * a;
  xn[3] = a + Ts * j;
  xn[4] = t1 + Ts * v / l1 * tan(dl);
  xn[5] = t2 + Ts * v / l2 * (sin(t1 - t2) - lh / l1 * cos(t1 - t2) * tan(dl));
  xn[6] = dl + Ts * w;
  xn[7] = x[7] + Ts * nu;
  for (int k = 0; k < 8; ++k) d.plant_x[k] = xn[k];
}

__global__ void k_plant(const SolveDesc* __restrict__ dp) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  plant_step(*dp);
}

// batched: one thread per instance, only those that asked for it
__global__ void k_plant_batch(const SolveDesc* __restrict__ descs, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (descs[i].flags & BRMPPI_ADVANCE_PLANT) plant_step(descs[i]);
}

// ---------------------------------------------------------------------------
// Debug: raw Philox blocks and the normals a rollout draws
// ---------------------------------------------------------------------------
__global__ void k_philox_dump(const uint32_t* __restrict__ ctr, uint32_t k0, uint32_t k1, uint32_t n,
                              uint32_t* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t r[4];
  philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1, r);
  for (int k = 0; k < 4; ++k) out[4 * i + k] = r[k];
}

__global__ void k_normals_dump(uint32_t seed_lo, uint32_t seed_hi, uint32_t instance,
                               const uint32_t* __restrict__ s_tau, uint32_t n, uint32_t K,
                               float* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t s = s_tau[2 * i], tau = s_tau[2 * i + 1];
  for (uint32_t b = 0; 4 * b < K; ++b) {
    uint32_t r[4];
    float e[4];
    philox4x32_10(s, tau, b, instance, seed_lo, seed_hi, r);
    box_muller4(r, e);
    for (uint32_t k = 0; k < 4 && 4 * b + k < K; ++k) out[(size_t)i * K + 4 * b + k] = e[k];
  }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int NOB, bool G>
static hipError_t launch_rollout_t(const SolveDesc* descs, const Tile* tiles, uint32_t n_tiles,
                                   BatchCounters* ctr, uint32_t grid, uint32_t block, hipStream_t stream) {
  hipLaunchKernelGGL((k_rollout<NOB, G>), dim3(grid), dim3(block), 0, stream, descs, tiles, n_tiles, ctr);
  return hipGetLastError();
}

hipError_t launch_rollout(int bucket, const SolveDesc* descs, const Tile* tiles, uint32_t n_tiles,
                          BatchCounters* ctr, uint32_t grid, uint32_t block, hipStream_t stream) {
  if (block == 0 || block > (uint32_t)kMaxBlock || (block % 64) != 0) return hipErrorInvalidValue;
  switch (bucket) {
    case 0: return launch_rollout_t<0, false>(descs, tiles, n_tiles, ctr, grid, block, stream);
    case 2: return launch_rollout_t<2, true>(descs, tiles, n_tiles, ctr, grid, block, stream);
    case 8: return launch_rollout_t<8, true>(descs, tiles, n_tiles, ctr, grid, block, stream);
    case 16: return launch_rollout_t<16, true>(descs, tiles, n_tiles, ctr, grid, block, stream);
    case 32: return launch_rollout_t<32, true>(descs, tiles, n_tiles, ctr, grid, block, stream);
    default: return hipErrorInvalidValue;
  }
}

template <int NOB, bool G>
static int occ_t(uint32_t block) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rollout<NOB, G>, (int)block, 0) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

int rollout_blocks_per_cu(int bucket, uint32_t block) {
  switch (bucket) {
    case 0: return occ_t<0, false>(block);
    case 2: return occ_t<2, true>(block);
    case 8: return occ_t<8, true>(block);
    case 16: return occ_t<16, true>(block);
    default: return occ_t<32, true>(block);
  }
}

hipError_t launch_weights(const SolveDesc* descs, const Item* items, uint32_t n_items, BatchCounters* ctr,
                          uint32_t grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_weights, dim3(grid), dim3(kWThreads), 0, stream, descs, items, n_items, ctr);
  return hipGetLastError();
}

hipError_t launch_reduce(const SolveDesc* descs, const Item* items, uint32_t n_items, BatchCounters* ctr,
                         uint32_t grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_reduce, dim3(grid), dim3(kWThreads), 0, stream, descs, items, n_items, ctr);
  return hipGetLastError();
}

hipError_t launch_plant(const SolveDesc* desc, hipStream_t stream) {
  hipLaunchKernelGGL(k_plant, dim3(1), dim3(64), 0, stream, desc);
  return hipGetLastError();
}

hipError_t launch_plant_batch(const SolveDesc* descs, uint32_t n, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_plant_batch, dim3((n + 63) / 64), dim3(64), 0, stream, descs, n);
  return hipGetLastError();
}

hipError_t launch_philox_dump(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t n, uint32_t* out,
                              hipStream_t stream) {
  const uint32_t b = 256, g = (n + b - 1) / b;
  if (g == 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox_dump, dim3(g), dim3(b), 0, stream, ctr, k0, k1, n, out);
  return hipGetLastError();
}

hipError_t launch_normals_dump(uint32_t seed_lo, uint32_t seed_hi, uint32_t instance, const uint32_t* s_tau,
                               uint32_t n, uint32_t K, float* out, hipStream_t stream) {
  const uint32_t b = 256, g = (n + b - 1) / b;
  if (g == 0) return hipSuccess;
  hipLaunchKernelGGL(k_normals_dump, dim3(g), dim3(b), 0, stream, seed_lo, seed_hi, instance, s_tau, n, K, out);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const uint32_t b = 256;
  const size_t g = (n + b - 1) / b;
  hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)g), dim3(b), 0, stream, p, value, n);
  return hipGetLastError();
}

}  // namespace brm
