// gfx950 kernels of one BR-MPPI control update (arXiv 2508.05773).
//
//   k_noise   : Philox4x32-10 + Box-Muller normals of every (sample, step)
//               in parallel (for the rollout variants that read them).
//   k_rollout : S rollouts of the tractor-trailer model, each step projected
//               onto the barrier-rate equalities (eq. (9)) with the
//               soft-bound closed form (eqs. (11)-(12)), contouring cost
//               (eqs. (13)-(15)) accumulated; writes the applied inputs
//               [3T][S] and the cost of every sample.  One or several lanes
//               per sample; noise drawn in the kernel or read from k_noise.
//   k_reduce  : weights exp(-(J - m)/lambda) (Sec. III-B) and the weighted
//               average of the applied inputs (eq. (5)) from HBM, in units of
//               32 samples and groups of 32 units merged by log-sum-exp; the
//               last block writes the new nominal sequence, the receding-
//               horizon shift and, on request, a closed-loop FP64 plant step
//               (eq. (6)).  A single-instance rollout whose tiles are whole
//               units does the same reduction itself from LDS (fused
//               epilogue): the applied inputs then never reach HBM.
//
// A sample's state, barrier rates and row terms stay in registers.  Obstacles
// (with their shape matrices) and a window of the path are staged in LDS per
// tile.  Positions are carried relative to the start position and progress
// relative to the start progress so that FP32 keeps sub-micrometre resolution
// far from the origin.
#include <math.h>

#include <type_traits>

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

// Box-Muller on the pairs (u0, u1) and (u2, u3): radius sqrt(-2 ln u0),
// angle 2 pi u1.  The uniforms lie in [2^-24, 1), so the hardware log2,
// square root, sine and cosine need none of the library's range reduction or
// special cases; the hardware sine and cosine take the angle in revolutions,
// so 2 pi u1 is never rounded.  Over all 2^23 uniforms the radius is within
// 4.9e-7 and the sine and cosine within 1.3e-7 of the exact values.
constexpr float kLn2 = 0.693147182f;
__device__ __forceinline__ float bm_radius(float u) {
  return __builtin_amdgcn_sqrtf(-2.0f * kLn2 * __builtin_amdgcn_logf(u));
}
__device__ __forceinline__ void box_muller4(const uint32_t r[4], float* n) {
  const float u0 = unif23(r[0]), u1 = unif23(r[1]), u2 = unif23(r[2]), u3 = unif23(r[3]);
  const float rad0 = bm_radius(u0), rad1 = bm_radius(u2);
  n[0] = rad0 * __builtin_amdgcn_cosf(u1);
  n[1] = rad0 * __builtin_amdgcn_sinf(u1);
  n[2] = rad1 * __builtin_amdgcn_cosf(u3);
  n[3] = rad1 * __builtin_amdgcn_sinf(u3);
}

constexpr float kTwoPi = 6.283185307179586f;
constexpr float kInvTwoPi = 0.15915494309189535f;

__device__ __forceinline__ float wrap_angle(float x) { return x - kTwoPi * rintf(x * kInvTwoPi); }

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Loads and stores through global-address-space pointers.  Pointers read from
// a descriptor are generic, and a generic (flat) access also counts against
// the LDS/scalar wait counter: every wait for an LDS or scalar result would
// then wait for the step-ahead HBM loads as well.
typedef float gvec4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float gld(const float* p) {
  return *(const __attribute__((address_space(1))) float*)p;
}
__device__ __forceinline__ float4 gld4(const float4* p) {
  const gvec4 v = *(const __attribute__((address_space(1))) gvec4*)p;
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gst(float* p, float v) { *(__attribute__((address_space(1))) float*)p = v; }
// LDS reads and writes through local-address-space pointers (and gst4, a
// 16-byte global store).  The instance merge is a function of its own, not
// inlined into the kernel, where a pointer argument is generic: a generic
// access to LDS compiles to a flat access, which is slower and counts against
// both wait counters.  Every pointer passed to the LDS helpers points into LDS.
typedef __attribute__((address_space(3))) float lds_float;
typedef __attribute__((address_space(3))) double lds_double;
typedef __attribute__((address_space(3))) gvec4 lds_vec4;
__device__ __forceinline__ float lds(const float* p) { return *(const lds_float*)p; }
__device__ __forceinline__ double lds(const double* p) { return *(const lds_double*)p; }
__device__ __forceinline__ float4 lds(const float4* p) {
  const gvec4 v = *(const lds_vec4*)p;
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void lds_put(float* p, float v) { *(lds_float*)p = v; }
__device__ __forceinline__ void lds_put(double* p, double v) { *(lds_double*)p = v; }
__device__ __forceinline__ void lds_put(float4* p, float4 v) {
  gvec4 w;
  w.x = v.x;
  w.y = v.y;
  w.z = v.z;
  w.w = v.w;
  *(lds_vec4*)p = w;
}
__device__ __forceinline__ void gst4(float4* p, float4 v) {
  gvec4 w;
  w.x = v.x;
  w.y = v.y;
  w.z = v.z;
  w.w = v.w;
  *(__attribute__((address_space(1))) gvec4*)p = w;
}

// GLB: through the global address space (the multi-lane forms, whose step has
// one wave per SIMD or so and nothing to hide a needless wait), or through the
// pointer as it is (the one-lane forms, whose register budget is the limit:
// the global forms let the compiler hoist loads and lengthen live ranges)
template <bool GLB>
__device__ __forceinline__ float ldf(const float* p) {
  if constexpr (GLB) return gld(p);
  else return *p;
}
template <bool GLB>
__device__ __forceinline__ void stf(float* p, float v) {
  if constexpr (GLB) gst(p, v);
  else *p = v;
}

// Per-lane choices inside the step are written as selects marked
// unpredictable, so that the compiler keeps them as lane selects instead of
// divergent branches (each of which costs exec-mask instructions and splits
// the step into separately scheduled regions).
__device__ __forceinline__ float sel(bool c, float a, float b) { return __builtin_unpredictable(c) ? a : b; }

// Obstacle row staged in LDS: the obstacle's centre relative to the tile
// origin, velocity; for e = 2 the shape matrix Q = R' diag((mx+r)^-2,
// (my+r)^-2) R of eq. (16); the rotation (co, so) into the obstacle frame and
// the per-axis coefficients k = (m+r)^-e (e4 = 1 for e = 4); the row's
// footprint disc (dA, dB).
struct ObsL {
  float cx, cy, vx, vy, q11, q12, q22, e4, co, so, k0, k1;
  float dA, dB;   // the row's footprint disc: centre p + dA e1 - dB f2
};

struct RefPoint {
  float x, y, th1, th2;
};

// Reference zeta(psi): linear interpolation between waypoints, headings by the
// wrapped difference, clamped to the ends.  f = phi0 + psi_rel/ds is the
// fractional waypoint index relative to k0.
template <bool GLB, bool SPLIT = false>
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
  const int li = gi - w0;
  float4 A, B;
  if constexpr (GLB && SPLIT) {
    // the window in LDS serves every lane unless one leaves it: then (a
    // wave-uniform, rare case) the lanes outside read their points from HBM.
    // LDS is read through the local address space and HBM through the global
    // one, each consumed on its own side of the branch: no flat access, whose
    // wait would also drain the step-ahead HBM loads in flight.
    const int lc = min(max(li, 0), nw - 2);
    const bool outside = !(li >= 0 && li + 1 < nw);
    A = lds(spath + lc);
    B = lds(spath + lc + 1);
    if (__any(outside)) {
      const float4 Ag = gld4(gpath + gi), Bg = gld4(gpath + gi + 1);
      A.x = outside ? Ag.x - ox : A.x;
      A.y = outside ? Ag.y - oy : A.y;
      A.z = outside ? Ag.z : A.z;
      A.w = outside ? Ag.w : A.w;
      B.x = outside ? Bg.x - ox : B.x;
      B.y = outside ? Bg.y - oy : B.y;
      B.z = outside ? Bg.z : B.z;
      B.w = outside ? Bg.w : B.w;
    }
  } else if constexpr (GLB) {
    // the same through a generic pointer (the eight-lane form's choice)
    const int lc = min(max(li, 0), nw - 2);
    const bool outside = !(li >= 0 && li + 1 < nw);
    if (__any(outside)) {
      const float4* pa = outside ? gpath + gi : spath + lc;
      A = pa[0];
      B = pa[1];
      const float dx = outside ? ox : 0.0f, dy = outside ? oy : 0.0f;
      A.x -= dx;
      A.y -= dy;
      B.x -= dx;
      B.y -= dy;
    } else {
      A = spath[lc];
      B = spath[lc + 1];
    }
  } else {
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
// Launch shapes: G lanes share one sample (G = 1, 2, 4, 8).  Every lane of a group
// carries the full state; obstacle o's barrier row is computed by group lane
// o % G, and the rows' projection terms are summed over the group by DPP
// butterflies in a canonical tree of eight virtual lanes (below), so that
// every lane ends with the same sums, bit for bit, as a one-lane sample.  With PRE the
// normals come from the noise buffer filled by k_noise (same Philox and
// Box-Muller code) instead of being drawn in the rollout.  Results are
// therefore bitwise identical for every (G, PRE) and block size.

struct ProjConst {
  float Ma, inv_Ma, amid, h_eps, W_a, rho;
};

// projection terms of one row of eq. (9) after eliminating its auxiliary
// input: (M_u + c g g') u = ... + c g rr, and the quantities the next barrier
// rate needs
struct RowTerms {
  float c, g0, g1, rr, Lf, ih;
};

__device__ __forceinline__ RowTerms row_terms(const ProjConst& K, float hhat, float Lf, float g0, float g1,
                                              float atil, float alpha) {
  const float ah = fabsf(hhat);
  const float hh = sel(ah < K.h_eps, sel(hhat < 0.0f, -K.h_eps, K.h_eps), hhat);
  const float b = -Lf - alpha * hh;
  const float abar = (K.W_a * atil + K.rho * (K.amid - alpha)) * K.inv_Ma;
  RowTerms R;
  R.rr = b - hh * abar;
  R.ih = rcp(hh);
  R.c = K.Ma * R.ih * R.ih;
  R.g0 = g0;
  R.g1 = g1;
  R.Lf = Lf;
  return R;
}

// Row sums of the 2x2 normal equations of the eliminated projection,
// accumulated in FP64: sum_i c_i g_i g_i' and sum_i c_i g_i rr_i
struct Acc5 {
  double N00, N01, N11, y0, y1;
};

__device__ __forceinline__ Acc5 acc_zero() { return Acc5{0.0, 0.0, 0.0, 0.0, 0.0}; }

__device__ __forceinline__ void acc_row(Acc5& A, const RowTerms& R) {
  const double cg0 = (double)R.c * (double)R.g0, cg1 = (double)R.c * (double)R.g1;
  A.N00 = fma(cg0, (double)R.g0, A.N00);
  A.N01 = fma(cg0, (double)R.g1, A.N01);
  A.N11 = fma(cg1, (double)R.g1, A.N11);
  A.y0 = fma(cg0, (double)R.rr, A.y0);
  A.y1 = fma(cg1, (double)R.rr, A.y1);
}

__device__ __forceinline__ Acc5 acc_add(const Acc5& a, const Acc5& b) {
  return Acc5{a.N00 + b.N00, a.N01 + b.N01, a.N11 + b.N11, a.y0 + b.y0, a.y1 + b.y1};
}

// obstacle row, eqs. (16)-(17) with e = 2: with q = d + Ts d_dot,
// hhat = q'Qq - 1 + Ts^2 d'Q d_ddot; Lf and g along f = Ts f_c, g = Ts g_c
struct ObsRow {
  float hhat, Lf, g0, g1;
};

__device__ __forceinline__ ObsRow obstacle_row(const ObsL& ob, float px, float py, float v, float a, float c1,
                                               float s1, float vkd, float sec2, float t, float Ts, float Ts2,
                                               float inv_l1) {
  const float dx = px - (ob.cx + ob.vx * t), dy = py - (ob.cy + ob.vy * t);
  const float ddx = v * c1 - ob.vx, ddy = v * s1 - ob.vy;
  const float v2kd = v * vkd;
  const float dddx = a * c1 - v2kd * s1, dddy = a * s1 + v2kd * c1;
  const float qx = dx + Ts * ddx, qy = dy + Ts * ddy;
  const float Qqx = ob.q11 * qx + ob.q12 * qy, Qqy = ob.q12 * qx + ob.q22 * qy;
  const float Qdx = ob.q11 * dx + ob.q12 * dy, Qdy = ob.q12 * dx + ob.q22 * dy;
  const float dQe1 = Qdx * c1 + Qdy * s1, dQe2 = Qdy * c1 - Qdx * s1;
  const float qQe1 = Qqx * c1 + Qqy * s1, qQe2 = Qqy * c1 - Qqx * s1;
  // gradient of hhat: position, speed, heading, time
  const float gpx = 2.0f * Qqx + Ts2 * (ob.q11 * dddx + ob.q12 * dddy);
  const float gpy = 2.0f * Qqy + Ts2 * (ob.q12 * dddx + ob.q22 * dddy);
  const float h_v = 2.0f * Ts * qQe1 + 2.0f * Ts2 * vkd * dQe2;
  const float h_th = 2.0f * Ts * v * qQe2 + Ts2 * (a * dQe2 - v2kd * dQe1);
  const float h_t = -(gpx * ob.vx + gpy * ob.vy);
  ObsRow R;
  R.hhat = qx * Qqx + qy * Qqy - 1.0f + Ts2 * (Qdx * dddx + Qdy * dddy);
  R.Lf = Ts * (v * (gpx * c1 + gpy * s1) + h_v * a + h_th * vkd + h_t);
  R.g0 = Ts * Ts2 * dQe1;                          // Ts d hhat/da
  R.g1 = Ts * Ts2 * v * v * sec2 * inv_l1 * dQe2;   // Ts d hhat/d delta
  return R;
}

// Super-ellipse row (e = 4), eqs. (16)-(17): h = k0 y0^4 + k1 y1^4 - 1 in the
// obstacle frame (y = R d).  Per axis the expansion hhat = h + Ts hd +
// Ts^2/2 hdd and its partials in y, y_dot and y_ddot (third derivatives of h
// included) are formed, then chained to the state through y_dot = v e1' - vo'
// and y_ddot = a e1' + v^2 kd e2' (primes: obstacle frame).
__device__ __forceinline__ ObsRow obstacle_row_e4(const ObsL& ob, float px, float py, float v, float a, float c1,
                                                  float s1, float vkd, float sec2, float t, float Ts, float Ts2,
                                                  float inv_l1) {
  const float co = ob.co, so = ob.so;
  const float dx = px - (ob.cx + ob.vx * t), dy = py - (ob.cy + ob.vy * t);
  const float y0 = co * dx + so * dy, y1 = -so * dx + co * dy;
  const float e10 = co * c1 + so * s1, e11 = -so * c1 + co * s1;   // R e1; R e2 = (-e11, e10)
  const float vo0 = co * ob.vx + so * ob.vy, vo1 = -so * ob.vx + co * ob.vy;
  const float v2kd = v * vkd;
  const float yd0 = v * e10 - vo0, yd1 = v * e11 - vo1;
  const float ydd0 = a * e10 - v2kd * e11, ydd1 = a * e11 + v2kd * e10;
  float hh[2], P[2], V[2], A[2];
  const float k[2] = {ob.k0, ob.k1}, y[2] = {y0, y1}, yd[2] = {yd0, yd1}, ydd[2] = {ydd0, ydd1};
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float y2 = y[i] * y[i], y3 = y2 * y[i];
    const float f1 = 4.0f * k[i] * y3, f2 = 12.0f * k[i] * y2, f3 = 24.0f * k[i] * y[i];
    const float hd = f1 * yd[i], hdd = f2 * yd[i] * yd[i] + f1 * ydd[i];
    hh[i] = k[i] * y2 * y2 + Ts * hd + 0.5f * Ts2 * hdd;
    P[i] = f1 + Ts * f2 * yd[i] + 0.5f * Ts2 * (f3 * yd[i] * yd[i] + f2 * ydd[i]);   // d hhat / d y
    V[i] = Ts * f1 + Ts2 * f2 * yd[i];                                             // d hhat / d y_dot
    A[i] = 0.5f * Ts2 * f1;                                                        // d hhat / d y_ddot
  }
  const float Ae1 = A[0] * e10 + A[1] * e11, Ae2 = -A[0] * e11 + A[1] * e10;
  const float Ve1 = V[0] * e10 + V[1] * e11, Ve2 = -V[0] * e11 + V[1] * e10;
  const float Pe1 = P[0] * e10 + P[1] * e11, Pvo = P[0] * vo0 + P[1] * vo1;
  const float h_v = Ve1 + 2.0f * vkd * Ae2;
  const float h_th = v * Ve2 + a * Ae2 - v2kd * Ae1;
  ObsRow R;
  R.hhat = hh[0] + hh[1] - 1.0f;
  R.Lf = Ts * (v * Pe1 + h_v * a + h_th * vkd - Pvo);
  R.g0 = Ts * Ae1;                                  // Ts d hhat/da
  R.g1 = Ts * v * v * sec2 * inv_l1 * Ae2;          // Ts d hhat/d delta
  return R;
}

// Kinematics of a footprint disc centre c = p + A e1 - B f2 along the drift
// (inputs zero), for the rows of a footprint other than the rear axle (Sec.
// IV-C): e1, e2 the tractor's heading and its left normal, f2, n2 the
// trailer's; every quantity is P0 + A PA - B PB with the step's parts below.
//   velocity  c'   = v e1 + A w1 e2 - B w2 n2
//   accel.    c''  = a e1 + v w1 e2 + A (w1' e2 - w1^2 e1) - B (w2' n2 - w2^2 f2)
//   jerk      c''' = -v w1^2 e1 + (2 a w1 + v w1') e2 + A (-3 w1 w1' e1 - w1^3 e2)
//                    + B (3 w2 w2' f2 + (w2^3 - w2'') n2)
// with w1 = th1', w2 = th2' of eq. (6) and their drift derivatives; and the
// partials through which the inputs act: dc'/d delta, dc''/da, dc''/d delta.
struct DiscBasis {
  float f2x, f2y;                                  // position: P0 = p, PA = e1, PB = f2
  float v0x, v0y, vAx, vAy, vBx, vBy;              // velocity
  float a0x, a0y, aAx, aAy, aBx, aBy;              // drift acceleration
  float j0x, j0y, jAx, jAy, jBx, jBy;              // drift jerk
  float gAx, gAy, gBx, gBy;                        // d velocity / d delta (P0 = 0)
  float ha0x, ha0y, haAx, haAy, haBx, haBy;        // d acceleration / d a
  float hd0x, hd0y, hdAx, hdAy, hdBx, hdBy;        // d acceleration / d delta
};

__device__ __forceinline__ DiscBasis disc_basis(float v, float a, float c1, float s1, float cp, float sp, float tn,
                                                float sec2, float inv_l1, float inv_l2, float ch) {
  DiscBasis D;
  const float e2x = -s1, e2y = c1;
  D.f2x = c1 * cp + s1 * sp;          // theta2 = theta1 - phi
  D.f2y = s1 * cp - c1 * sp;
  const float n2x = -D.f2y, n2y = D.f2x;
  const float kd = tn * inv_l1, dkd = sec2 * inv_l1;
  const float W = inv_l2 * (sp - ch * cp * tn);             // w2 = v W
  const float Wp = inv_l2 * (cp + ch * sp * tn);            // dW/dphi (d2W/dphi2 = -W)
  const float Wd = -inv_l2 * ch * cp * sec2;                // dW/d delta
  const float Wpd = inv_l2 * ch * sp * sec2;                // d2W/dphi d delta
  const float w1 = v * kd, w2 = v * W, ph = w1 - w2;
  const float w1d = a * kd;                                 // w1' along the drift
  const float w2d = a * W + v * Wp * ph;                    // w2'
  const float w2dd = 2.0f * a * Wp * ph - v * W * ph * ph + v * Wp * (w1d - w2d);   // w2''
  D.v0x = v * c1;  D.v0y = v * s1;
  D.vAx = w1 * e2x;  D.vAy = w1 * e2y;
  D.vBx = w2 * n2x;  D.vBy = w2 * n2y;
  D.a0x = a * c1 + v * w1 * e2x;  D.a0y = a * s1 + v * w1 * e2y;
  D.aAx = w1d * e2x - w1 * w1 * c1;  D.aAy = w1d * e2y - w1 * w1 * s1;
  D.aBx = w2d * n2x - w2 * w2 * D.f2x;  D.aBy = w2d * n2y - w2 * w2 * D.f2y;
  const float j1 = -v * w1 * w1, j2 = 2.0f * a * w1 + v * w1d;
  D.j0x = j1 * c1 + j2 * e2x;  D.j0y = j1 * s1 + j2 * e2y;
  const float jA1 = -3.0f * w1 * w1d, jA2 = -w1 * w1 * w1;
  D.jAx = jA1 * c1 + jA2 * e2x;  D.jAy = jA1 * s1 + jA2 * e2y;
  const float jB1 = -3.0f * w2 * w2d, jB2 = w2dd - w2 * w2 * w2;
  D.jBx = jB1 * D.f2x + jB2 * n2x;  D.jBy = jB1 * D.f2y + jB2 * n2y;
  D.gAx = v * dkd * e2x;  D.gAy = v * dkd * e2y;
  D.gBx = v * Wd * n2x;  D.gBy = v * Wd * n2y;
  D.ha0x = c1;  D.ha0y = s1;
  D.haAx = kd * e2x;  D.haAy = kd * e2y;
  D.haBx = W * n2x;  D.haBy = W * n2y;
  const float w2d_dl = a * Wd + v * Wpd * ph + v * Wp * (v * dkd - v * Wd);
  D.hd0x = v * v * dkd * e2x;  D.hd0y = v * v * dkd * e2y;
  D.hdAx = a * dkd * e2x - 2.0f * w1 * v * dkd * c1;  D.hdAy = a * dkd * e2y - 2.0f * w1 * v * dkd * s1;
  D.hdBx = w2d_dl * n2x - 2.0f * w2 * v * Wd * D.f2x;  D.hdBy = w2d_dl * n2y - 2.0f * w2 * v * Wd * D.f2y;
  return D;
}

// Row of an obstacle around a footprint disc (e = 2 or 4), eqs. (16)-(17):
// per axis of the obstacle frame (y = R (c - p_o(t)), k = (m + r)^-e)
// h = sum k y^e - 1 and its time derivatives along the drift from those of
// y; hhat = h + Ts hd + Ts^2/2 hdd; Lf = Ts d hhat/dt along the drift
// (obstacle motion included) = Ts (hd + Ts hdd + Ts^2/2 hddd); g = Ts (d
// hhat/da, d hhat/d delta), which reach hhat through c' (delta) and c''.
__device__ __forceinline__ ObsRow obstacle_row_disc(const ObsL& ob, const DiscBasis& D, float px, float py,
                                                    float c1, float s1, float t, float Ts, float Ts2) {
  const float A = ob.dA, B = ob.dB;
  const float dx = px + A * c1 - B * D.f2x - (ob.cx + ob.vx * t);
  const float dy = py + A * s1 - B * D.f2y - (ob.cy + ob.vy * t);
  const float ux = D.v0x + A * D.vAx - B * D.vBx - ob.vx, uy = D.v0y + A * D.vAy - B * D.vBy - ob.vy;
  const float wx = D.a0x + A * D.aAx - B * D.aBx, wy = D.a0y + A * D.aAy - B * D.aBy;
  const float zx = D.j0x + A * D.jAx - B * D.jBx, zy = D.j0y + A * D.jAy - B * D.jBy;
  const float gx = A * D.gAx - B * D.gBx, gy = A * D.gAy - B * D.gBy;
  const float hax = D.ha0x + A * D.haAx - B * D.haBx, hay = D.ha0y + A * D.haAy - B * D.haBy;
  const float hdx = D.hd0x + A * D.hdAx - B * D.hdBx, hdy = D.hd0y + A * D.hdAy - B * D.hdBy;
  const float co = ob.co, so = ob.so;
  const float y[2] = {co * dx + so * dy, -so * dx + co * dy};
  const float yd[2] = {co * ux + so * uy, -so * ux + co * uy};
  const float ydd[2] = {co * wx + so * wy, -so * wx + co * wy};
  const float yddd[2] = {co * zx + so * zy, -so * zx + co * zy};
  const float ydl[2] = {co * gx + so * gy, -so * gx + co * gy};          // d y_dot / d delta
  const float ya[2] = {co * hax + so * hay, -so * hax + co * hay};       // d y_ddot / da
  const float yddl[2] = {co * hdx + so * hdy, -so * hdx + co * hdy};     // d y_ddot / d delta
  const bool e4 = ob.e4 != 0.0f;
  const float k[2] = {ob.k0, ob.k1};
  float h = -1.0f, hd = 0.0f, hdd = 0.0f, hddd = 0.0f, da = 0.0f, dd1 = 0.0f, dd2 = 0.0f;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float yy = y[i] * y[i];
    // derivatives of k y^e: (f0, f1, f2, f3)
    const float f0 = sel(e4, k[i] * yy * yy, k[i] * yy);
    const float f1 = sel(e4, 4.0f * k[i] * yy * y[i], 2.0f * k[i] * y[i]);
    const float f2 = sel(e4, 12.0f * k[i] * yy, 2.0f * k[i]);
    const float f3 = sel(e4, 24.0f * k[i] * y[i], 0.0f);
    h += f0;
    hd += f1 * yd[i];
    hdd += f2 * yd[i] * yd[i] + f1 * ydd[i];
    hddd += f3 * yd[i] * yd[i] * yd[i] + 3.0f * f2 * yd[i] * ydd[i] + f1 * yddd[i];
    da += f1 * ya[i];
    dd1 += f1 * ydl[i];
    dd2 += 2.0f * f2 * yd[i] * ydl[i] + f1 * yddl[i];
  }
  ObsRow R;
  R.hhat = h + Ts * hd + 0.5f * Ts2 * hdd;
  R.Lf = Ts * (hd + Ts * hdd + 0.5f * Ts2 * hddd);
  R.g0 = Ts * (0.5f * Ts2 * da);
  R.g1 = Ts * (Ts * dd1 + 0.5f * Ts2 * dd2);
  return R;
}

// E4: the instance has super-ellipse obstacles (decided once per tile, so that
// ellipse-only instances run a step loop without the e = 4 code)
template <bool E4>
__device__ __forceinline__ ObsRow obstacle_row_any(const ObsL& ob, float px, float py, float v, float a, float c1,
                                                   float s1, float vkd, float sec2, float t, float Ts, float Ts2,
                                                   float inv_l1) {
  if (E4 && ob.e4 != 0.0f) return obstacle_row_e4(ob, px, py, v, a, c1, s1, vkd, sec2, t, Ts, Ts2, inv_l1);
  return obstacle_row(ob, px, py, v, a, c1, s1, vkd, sec2, t, Ts, Ts2, inv_l1);
}

// the row of obstacle slot `ob`: at the rear axle (e = 2, or 4 with E4) or,
// with DISC, around the slot's footprint disc
template <bool E4, bool DISC>
__device__ __forceinline__ ObsRow obstacle_row_sel(const ObsL& ob, const DiscBasis& D, float px, float py, float v,
                                                   float a, float c1, float s1, float vkd, float sec2, float t,
                                                   float Ts, float Ts2, float inv_l1) {
  if constexpr (DISC) {
    return obstacle_row_disc(ob, D, px, py, c1, s1, t, Ts, Ts2);
  } else {
    return obstacle_row_any<E4>(ob, px, py, v, a, c1, s1, vkd, sec2, t, Ts, Ts2, inv_l1);
  }
}

// value held by lane Q of each G-lane group, broadcast to the group (DPP quad
// permute; G = 2 or 4 divides a quad, G = 8 groups hold two quads that each
// carry the value)
template <int G, int Q>
__device__ __forceinline__ float group_bcast(float x) {
  if constexpr (G == 1) {
    return x;
  } else {
    constexpr int ctrl = (G >= 4) ? (Q * 0x55) : ((Q) | (Q << 2) | ((2 + Q) << 4) | ((2 + Q) << 6));
    // every lane reads an in-range lane of its own quad: no "old" value needed
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), ctrl, 0xF, 0xF, true));
  }
}

// DPP controls of the three butterfly levels over 8 lanes: lane i reads lane
// i ^ 1, i ^ 2 (quad permutes), then 7 - i (half-row mirror: the other quad)
constexpr int kDppXor1 = 0xB1;
constexpr int kDppXor2 = 0x4E;
constexpr int kDppHalfMirror = 0x141;

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  const int lo2 = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, true);
  const int hi2 = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi2, lo2);
}

template <int CTRL>
__device__ __forceinline__ Acc5 acc_partner_add(const Acc5& a) {
  return acc_add(a, Acc5{dpp_f64<CTRL>(a.N00), dpp_f64<CTRL>(a.N01), dpp_f64<CTRL>(a.N11), dpp_f64<CTRL>(a.y0),
                         dpp_f64<CTRL>(a.y1)});
}

// Canonical accumulation order of the projection rows, independent of the
// number G of lanes per sample: row r belongs to virtual lane v(r) (hitch row
// k -> v = k, obstacle o -> v = o mod 8); a virtual lane sums its rows from
// zero in row order (hitch row first, then obstacles v, v + 8, ...); the 8
// virtual sums are added by a fixed binary tree (v ^ 1, then v ^ 2, then v ^ 4).
// Lane q of a group owns virtual lanes q + G i.  The levels that pair virtual
// lanes on different lanes run as DPP butterflies (IEEE addition commutes, so
// both partners hold the same bits), the rest inside the lane.
template <int G>
__device__ __forceinline__ Acc5 cross_lane_levels(Acc5 a) {
  if constexpr (G >= 2) a = acc_partner_add<kDppXor1>(a);
  if constexpr (G >= 4) a = acc_partner_add<kDppXor2>(a);
  if constexpr (G >= 8) a = acc_partner_add<kDppHalfMirror>(a);
  return a;
}

template <int G, int LO, int N, typename Leaf>
__device__ __forceinline__ Acc5 virtual_tree(Leaf& leaf) {
  if constexpr (N == 1) {
    return cross_lane_levels<G>(leaf(std::integral_constant<int, LO>{}));
  } else {
    const Acc5 l = virtual_tree<G, LO, N / 2>(leaf);
    const Acc5 r = virtual_tree<G, LO + N / 2, N / 2>(leaf);
    return acc_add(l, r);
  }
}

// Collision-penalty baseline (the paper's second MPPI baseline, Sec. V; its
// form is not given): sum over the obstacle rows of max(0, -h)^2 with h the
// obstacle function of eq. (16) (e = 2 or 4) at the row's point (the rear
// axle, or with DISC its footprint disc centre) and the current time, in row
// order (every lane of a group sums all rows).
template <bool E4, bool DISC>
__device__ __forceinline__ float collision_pen(const ObsL* __restrict__ sobs, int n_obs, float px, float py,
                                               float th1, float th2, float t) {
  float c1 = 0.0f, s1 = 0.0f, c2 = 0.0f, s2 = 0.0f;
  if constexpr (DISC) {
    sincosf(th1, &s1, &c1);
    sincosf(th2, &s2, &c2);
  }
  float pen = 0.0f;
  for (int o = 0; o < n_obs; ++o) {
    const ObsL ob = sobs[o];
    float qx = px, qy = py;
    if constexpr (DISC) {
      qx = px + ob.dA * c1 - ob.dB * c2;
      qy = py + ob.dA * s1 - ob.dB * s2;
    }
    const float dx = qx - (ob.cx + ob.vx * t), dy = qy - (ob.cy + ob.vy * t);
    float h;
    if (E4 && ob.e4 != 0.0f) {
      const float y0 = ob.co * dx + ob.so * dy, y1 = -ob.so * dx + ob.co * dy;
      const float z0 = y0 * y0, z1 = y1 * y1;
      h = ob.k0 * z0 * z0 + ob.k1 * z1 * z1 - 1.0f;
    } else {
      h = dx * (ob.q11 * dx + ob.q12 * dy) + dy * (ob.q12 * dx + ob.q22 * dy) - 1.0f;
    }
    pen += (h < 0.0f) ? h * h : 0.0f;
  }
  return pen;
}

// sine and cosine of the four angles a step needs (th1, th1 - th2, delta and
// the reference heading), one pair per lane for G >= 4, then broadcast.  The
// hardware sine and cosine (absolute error of order 1e-6 over the angles a
// rollout reaches) keep the library's range reduction off the step's chain.
struct StepTrig {
  float s1, c1, sp, cp, sd, cd, sr, cr;
};

__device__ __forceinline__ void step_sincos(float x, float* s, float* c) {
  *s = __sinf(x);
  *c = __cosf(x);
}

template <int G>
__device__ __forceinline__ StepTrig step_trig(int g, float a0, float a1, float a2, float a3) {
  StepTrig t;
  if constexpr (G == 1) {
    step_sincos(a0, &t.s1, &t.c1);
    step_sincos(a1, &t.sp, &t.cp);
    step_sincos(a2, &t.sd, &t.cd);
    step_sincos(a3, &t.sr, &t.cr);
  } else if constexpr (G == 2) {
    // lane g: angles g and g + 2
    float s0, c0, s2, c2;
    step_sincos(g == 0 ? a0 : a1, &s0, &c0);
    step_sincos(g == 0 ? a2 : a3, &s2, &c2);
    t.s1 = group_bcast<2, 0>(s0);
    t.c1 = group_bcast<2, 0>(c0);
    t.sp = group_bcast<2, 1>(s0);
    t.cp = group_bcast<2, 1>(c0);
    t.sd = group_bcast<2, 0>(s2);
    t.cd = group_bcast<2, 0>(c2);
    t.sr = group_bcast<2, 1>(s2);
    t.cr = group_bcast<2, 1>(c2);
  } else {
    // lane g of every quad: angle g mod 4
    const bool odd = (g & 1) != 0, high = (g & 2) != 0;
    const float a = sel(high, sel(odd, a3, a2), sel(odd, a1, a0));
    float sa, ca;
    step_sincos(a, &sa, &ca);
    t.s1 = group_bcast<G, 0>(sa);
    t.c1 = group_bcast<G, 0>(ca);
    t.sp = group_bcast<G, 1>(sa);
    t.cp = group_bcast<G, 1>(ca);
    t.sd = group_bcast<G, 2>(sa);
    t.cd = group_bcast<G, 2>(ca);
    t.sr = group_bcast<G, 3>(sa);
    t.cr = group_bcast<G, 3>(ca);
  }
  return t;
}

// Tracking part of eq. (13) with the reference heading's sine and cosine given.
__device__ __forceinline__ float tracking_cost_sc(const brmppi_params& P, const RefPoint& rf, float sr, float cr,
                                                  float px, float py, float th1, float th2) {
  const float ex = px - rf.x, ey = py - rf.y;
  const float ec = sr * ex - cr * ey;
  const float el = -cr * ex - sr * ey;
  const float e1 = wrap_angle(th1 - rf.th1);
  const float e2 = wrap_angle(th2 - rf.th2);
  return P.Qc * ec * ec + P.Ql * el * el + P.Qth1 * e1 * e1 + P.Qth2 * e2 * e2;
}

// Stage cost r(x, u*, psi) of eq. (13): tracking terms, effort on (j, omega)
// and the progress term mu (nu_bar - nu)^2.
__device__ __forceinline__ float stage_cost(const brmppi_params& P, const RefPoint& rf, float sr, float cr, float px,
                                            float py, float th1, float th2, float uj, float uw, float unu) {
  const float prog = P.nu_bar - unu;
  return tracking_cost_sc(P, rf, sr, cr, px, py, th1, th2) + P.R_j * uj * uj + P.R_w * uw * uw +
         P.mu * prog * prog;
}

// value held by lane Q of each G-lane group, correct in the group's lane 0
// (G = 8: lanes 4..7 hold it after a quad permute, and lane 0 reads lane 7
// through the half-row mirror)
template <int G, int Q>
__device__ __forceinline__ float lane_value(float x) {
  if constexpr (G < 8 || Q < 4) {
    return group_bcast<G, Q>(x);
  } else {
    const float y = group_bcast<4, Q - 4>(x);
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(y), kDppHalfMirror, 0xF, 0xF, true));
  }
}

// One sample's rollout over T steps, run by the G lanes of its group (lane g).
// Rows: every lane computes the hitch row g mod 2 (G = 1: both), obstacle o is
// computed by lane o mod G in its slot o / G.  After the projection every lane
// holds the same inputs, state and cost.
// s_u / s_J (fused epilogue): the tile's applied inputs [3T][lds_stride] and
// costs in LDS, at column t_local.
template <int NOB, bool GUIDED, int G, bool PRE, bool E4, bool DISC>
__device__ __forceinline__ void rollout_sample(const SolveDesc& d, uint32_t s, bool store, int g, const float* x0,
                                               const ObsL* __restrict__ sobs, const float4* __restrict__ spath,
                                               const float* __restrict__ s_un, int w0, int nw, int k0, float phi0,
                                               float* s_u, uint32_t lds_stride, uint32_t t_local, float* s_J) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8, "lanes per sample");
  static_assert(PRE || G == 1, "a sample shared by lanes reads precomputed normals");
  constexpr int NSL = GUIDED ? (NOB + G - 1) / G : 1;   // obstacle slots of this lane
  constexpr int NV = 8 / G;                            // virtual lanes of this lane
  constexpr int NH = (G == 1) ? 2 : 1;                 // hitch rows computed by this lane
  constexpr int NBMAX = GUIDED ? (5 + NOB + 3) / 4 : 1;  // Philox blocks (fused noise)
  // a copy: the compiler keeps the parameters in registers instead of
  // re-reading the descriptor (a scalar load and a wait) inside the step
  brmppi_params P = d.prm;
  float t0 = d.t0, inv_ds = d.inv_ds;
  float Ts = P.Ts, Ts2 = P.Ts * P.Ts;
  float inv_l1 = 1.0f / P.l1, inv_l2 = 1.0f / P.l2, ch = P.lh / P.l1;
  const int n_obs = (int)d.n_obs;
  const bool hitch = !(d.flags & BRMPPI_HITCH_OFF);
  // an unguided instance may share a guided launch: the flag is honoured here
  const bool guided = GUIDED && !(d.flags & BRMPPI_GUIDANCE_OFF);
  const bool penalty = (d.flags & BRMPPI_COLLISION_PENALTY) != 0;
  const int nb = guided ? (5 + n_obs + 3) / 4 : 1;
  const float ox = x0[0], oy = x0[1];
  const float4* __restrict__ gpath = d.path;
  const int n_path = (int)d.n_path;
  const int hk0 = (G == 1) ? 0 : (g & 1);    // first hitch row of this lane

  // soft-bound projection constants, eq. (11): M = W + rho I,
  // p = W z_des + rho/2 (lo + hi)
  ProjConst K;
  K.Ma = P.W_a + P.rho;
  K.inv_Ma = 1.0f / K.Ma;
  K.amid = 0.5f * (P.alpha_lo + P.alpha_hi);
  K.h_eps = P.h_eps;
  K.W_a = P.W_a;
  K.rho = P.rho;
  float Mj = P.W_j + P.rho, Mw = P.W_w + P.rho;
  float pj0 = 0.5f * P.rho * (P.j_lo + P.j_hi);
  float pw0 = 0.5f * P.rho * (P.w_lo + P.w_hi);
  if constexpr (G == 8) {
    // The eight-lane form has vector registers to spare (one wave per SIMD)
    // and too few scalar ones: the step's constants are held in vector
    // registers (an empty asm makes each a per-lane value), which frees the
    // scalar registers that were spilled to vector lanes and re-read in
    // every step, and saves the copies a scalar operand needs when an
    // instruction already reads one.
    auto vpin = [](float& x) { asm volatile("" : "+v"(x)); };
    vpin(P.sigma_j); vpin(P.sigma_w); vpin(P.sigma_nu); vpin(P.sigma_a);
    vpin(P.W_j); vpin(P.W_w); vpin(P.dtheta_max); vpin(P.kappa);
    vpin(P.Qc); vpin(P.Ql); vpin(P.Qth1); vpin(P.Qth2); vpin(P.R_j); vpin(P.R_w); vpin(P.mu); vpin(P.nu_bar);
    vpin(P.w_col); vpin(t0); vpin(inv_ds); vpin(Ts); vpin(Ts2); vpin(inv_l1); vpin(inv_l2); vpin(ch);
    vpin(K.Ma); vpin(K.inv_Ma); vpin(K.amid); vpin(K.h_eps); vpin(K.W_a); vpin(K.rho);
    vpin(Mj); vpin(Mw); vpin(pj0); vpin(pw0);
  }

  float px = 0.0f, py = 0.0f, v = x0[2], a = x0[3], th1 = x0[4], th2 = x0[5], dl = x0[6], psi = 0.0f;
  float alpha_h[NH];
#pragma unroll
  for (int k = 0; k < NH; ++k) alpha_h[k] = P.alpha0;
  float alpha_o[NSL];
#pragma unroll
  for (int j = 0; j < NSL; ++j) alpha_o[j] = P.alpha0;
  double J = 0.0;
  const uint32_t S_pad = d.S_pad;
  float* __restrict__ ustar = d.u_star;
  const float* __restrict__ unom = d.u_nom_in;
  constexpr bool kGlb = (G > 1);
  // Two arrangements of the step's memory accesses, each the faster for its
  // forms (measured):
  // - eight lanes per sample (few samples: one wave per SIMD, every latency
  //   exposed, the schedule of the step's chain what counts): the next step's
  //   nominal inputs fetched from HBM one step ahead, the normals' queue slot
  //   refilled as soon as it is read;
  // - the others (several waves per SIMD, memory waits what counts): the
  //   nominal inputs read from LDS (staged with the tile), the slot refilled
  //   after the last use of its values, whole pairs of steps per pass of the
  //   loop, the reference window read without flat accesses.
  constexpr bool kAhead = (G == 8);
  constexpr bool kLate = PRE && !kAhead;
  // Stage costs.  One lane per sample evaluates the cost of every step.  With
  // G > 1 lanes the cost is not repeated on every lane: lane g keeps the cost
  // inputs of the steps tau with tau % G == g (state, progress and applied
  // inputs), and once per G steps each lane evaluates the cost of its kept
  // step, reference lookup included; lane 0 then adds the G costs to J in step
  // order.  J therefore receives the same terms in the same order as in the
  // one-lane form, and only lane 0 (the lane that stores) holds it.
  constexpr bool kBatchCost = (G > 1);
  RefPoint rf{};
  if constexpr (!kBatchCost) rf = reference<kGlb, !kAhead>(phi0 + psi * inv_ds, k0, n_path, spath, w0, nw, gpath, ox, oy);
  float k_px = 0.0f, k_py = 0.0f, k_th1 = 0.0f, k_th2 = 0.0f, k_psi = 0.0f, k_uj = 0.0f, k_uw = 0.0f, k_unu = 0.0f;
  float un_j = 0.0f, un_w = 0.0f, un_nu = 0.0f;
  if constexpr (kAhead) {
    un_j = ldf<kGlb>(unom + 0);
    un_w = ldf<kGlb>(unom + 1);
    un_nu = ldf<kGlb>(unom + 2);
  }
  // the hitch rows are owned by lanes 0 and 1; the others zero their copy by
  // this factor (c = 0 makes every term of the row's sums an exact zero)
  const float hz_own = (hitch && g < 2) ? 1.0f : 0.0f;

  // Precomputed normals are loaded PF = 2 steps ahead into a queue of two
  // slots: step tau reads slot tau % 2 and refills it with step tau + 2.  The
  // loop is unrolled by two so that the slot is a compile-time index (no
  // register moves, which would wait for the loads in flight).  Every load is
  // in range (step and row indices clamped), so none needs a branch; rows
  // past the instance's own (obstacles o >= n_obs, unguided instances) feed
  // only rows whose terms are zeroed or unused.
  static_assert(!PRE || kNoisePrefetch == 2, "two queue slots");
  constexpr int PF = PRE ? 2 : 1;
  float nx_in[PF][3], nx_h[PF][NH], nx_o[PF][NSL];
  const uint32_t n_rows = d.n_normals;
  const size_t step_stride = (size_t)n_rows * S_pad;
  auto load_normals = [&](uint32_t tau, int q) {
    if constexpr (PRE) {
      const float* __restrict__ base = d.noise + (size_t)tau * step_stride + s;
#pragma unroll
      for (int k = 0; k < 3; ++k) nx_in[q][k] = ldf<kGlb>(base + (size_t)k * S_pad);
#pragma unroll
      for (int k = 0; k < NH; ++k)
        nx_h[q][k] = ldf<kGlb>(base + (size_t)min((uint32_t)(3 + hk0 + k), n_rows - 1) * S_pad);
#pragma unroll
      for (int j = 0; j < NSL; ++j)
        nx_o[q][j] = ldf<kGlb>(base + (size_t)min((uint32_t)(5 + g + G * j), n_rows - 1) * S_pad);
    }
  };
  if constexpr (PRE) {
    // (kLate: slot 0 before slot 1, in this order, as inside the loop)
    load_normals(0u, 0);
    if constexpr (kLate) __builtin_amdgcn_sched_barrier(0);
    load_normals(min(1u, d.T - 1), 1);
    if constexpr (kLate) __builtin_amdgcn_sched_barrier(0);
  }

  auto step = [&](const uint32_t tau, auto SLOT) __attribute__((always_inline)) {
    constexpr int q = decltype(SLOT)::value;
    // --- noise: normals 0..2 perturb the inputs, 3 and 4 the hitch rows'
    // auxiliary inputs, 5 + o obstacle o's ---
    float e_in[3], e_h[NH], e_o[NSL];
    if constexpr (PRE) {
#pragma unroll
      for (int k = 0; k < 3; ++k) e_in[k] = nx_in[q][k];
#pragma unroll
      for (int k = 0; k < NH; ++k) e_h[k] = nx_h[q][k];
#pragma unroll
      for (int j = 0; j < NSL; ++j) e_o[j] = nx_o[q][j];
      if constexpr (!kLate) load_normals(min(tau + 2, d.T - 1), q);
    } else {
      float eps[4 * NBMAX];
#pragma unroll
      for (int b = 0; b < NBMAX; ++b) {
        if (b < nb) {
          uint32_t r[4];
          philox4x32_10(s, tau, (uint32_t)b, d.instance, d.seed_lo, d.seed_hi, r);
          box_muller4(r, &eps[4 * b]);
        }
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) e_in[k] = eps[k];
      if constexpr (GUIDED) {
#pragma unroll
        for (int k = 0; k < NH; ++k) e_h[k] = eps[3 + k];
#pragma unroll
        for (int j = 0; j < NSL; ++j) e_o[j] = eps[5 + j];   // G == 1: slot j is obstacle j
      }
    }
    float uj, uw, unu;
    if constexpr (kAhead) {
      uj = un_j + P.sigma_j * e_in[0];
      uw = un_w + P.sigma_w * e_in[1];
      unu = un_nu + P.sigma_nu * e_in[2];
      const uint32_t tn = min(tau + 1, d.T - 1);
      un_j = ldf<kGlb>(unom + 3 * tn + 0);
      un_w = ldf<kGlb>(unom + 3 * tn + 1);
      un_nu = ldf<kGlb>(unom + 3 * tn + 2);
    } else {
      // staged in LDS with the tile: a broadcast read, no HBM load to keep in
      // flight across the loop's back edge
      uj = lds(s_un + 3 * tau + 0) + P.sigma_j * e_in[0];
      uw = lds(s_un + 3 * tau + 1) + P.sigma_w * e_in[1];
      unu = lds(s_un + 3 * tau + 2) + P.sigma_nu * e_in[2];
    }
    // the rows' auxiliary-input perturbations: with the inputs' above, the
    // only uses of the step's normals (kLate: formed here, before the refill;
    // otherwise in the rows)
    float at_h[NH], at_o[NSL];
    if constexpr (GUIDED && kLate) {
#pragma unroll
      for (int k = 0; k < NH; ++k) at_h[k] = P.sigma_a * e_h[k];
#pragma unroll
      for (int j = 0; j < NSL; ++j) at_o[j] = P.sigma_a * e_o[j];
    }
    const float psi_next = psi + Ts * unu;
    if constexpr (!kBatchCost) {
      if (tau > 0) rf = reference<kGlb, !kAhead>(phi0 + psi * inv_ds, k0, n_path, spath, w0, nw, gpath, ox, oy);
    }
    // (the fourth angle, the reference heading, only for the per-step cost)
    const StepTrig tg = step_trig<G>(g, th1, th1 - th2, dl, kBatchCost ? dl : rf.th1);
    const float s1 = tg.s1, c1 = tg.c1, sp = tg.sp, cp = tg.cp;
    const float tn = tg.sd * rcp(tg.cd);    // |delta| stays far from pi/2: cos > 0
    const float kd = tn * inv_l1;     // th1_dot = v kd
    const float vkd = v * kd;
    const float Aw2 = sp - ch * cp * tn;
    // Refill the queue slot with step tau + 2 only now, after the last use of
    // its values (the trigonometry above covers the nominal inputs' LDS
    // read): a refill hoisted above a use needs a second register, and the
    // copy back into the slot's register at the loop's back edge would wait
    // for every load in flight (the prefetch lost).  The empty asm pins the
    // normals' products here (the compiler would otherwise sink them to their
    // uses in the rows, past the refill) and the scheduling barrier keeps the
    // refill below them.
    if constexpr (kLate) {
      asm volatile("" : "+v"(uj), "+v"(uw), "+v"(unu));
      if constexpr (GUIDED) {
#pragma unroll
        for (int k = 0; k < NH; ++k) asm volatile("" : "+v"(at_h[k]));
#pragma unroll
        for (int j = 0; j < NSL; ++j) asm volatile("" : "+v"(at_o[j]));
      }
      __builtin_amdgcn_sched_barrier(0);
      load_normals(min(tau + 2, d.T - 1), q);
    }

    if (GUIDED && guided) {
      const float sec2 = 1.0f + tn * tn;
      const float t = t0 + (float)tau * Ts;
      DiscBasis DB;
      if constexpr (DISC) DB = disc_basis(v, a, c1, s1, cp, sp, tn, sec2, inv_l1, inv_l2, ch);

      // hitch rows, eq. (18) split into h_s = dth_max - kappa v + s (th1 - th2),
      // first-order expansion hhat = h + Ts hd
      // (with G > 1 lanes the rows are formed whether the instance has them or
      // not, and zeroed by hz_own: no branch in the step)
      RowTerms H[NH];
      if (G > 1 || hitch) {
        const float D = v * inv_l2 * Aw2 - vkd;                 // th2_dot - th1_dot
        const float D_v = inv_l2 * Aw2 - kd;
        const float D_phi = v * inv_l2 * (cp + ch * sp * tn);
        const float D_dl = -v * sec2 * (inv_l2 * ch * cp + inv_l1);
        const float phi = th1 - th2;
#pragma unroll
        for (int k = 0; k < NH; ++k) {
          const float sg = (hk0 + k) == 0 ? 1.0f : -1.0f;
          const float h = P.dtheta_max - P.kappa * v + sg * phi;
          const float hd = -P.kappa * a - sg * D;
          const float hv = -P.kappa - sg * Ts * D_v;
          const float Lf = Ts * (hv * a - sg * (1.0f - Ts * D_phi) * D);
          H[k] = row_terms(K, h + Ts * hd, Lf, -P.kappa * Ts2, -sg * Ts2 * D_dl,
                         kLate ? at_h[k] : P.sigma_a * e_h[k], alpha_h[k]);
        }
      }
      // rows of virtual lane g + G i: its hitch row, then obstacles in order
      RowTerms O[NSL];
      auto leaf = [&](auto I) -> Acc5 {
        constexpr int i = decltype(I)::value;
        const int vl = g + G * i;
        Acc5 A = acc_zero();
        if constexpr (G == 1) {
          if (hitch && vl < 2) acc_row(A, H[vl]);
        } else if (i == 0) {
          // lanes 0 and 1 hold the hitch rows; the others add exact zeros (c =
          // 0 and finite g, rr give products of +-0, and an accumulator is
          // never -0, so x + 0 keeps its bits)
          RowTerms Hz = H[0];
          Hz.c *= hz_own;
          acc_row(A, Hz);
        }
#pragma unroll
        for (int j = i; j < NSL; j += NV) {
          const int o = g + G * j;
          if constexpr (G == 1) {
            if (o < n_obs) {
              const ObsRow R = obstacle_row_sel<E4, DISC>(sobs[o], DB, px, py, v, a, c1, s1, vkd, sec2, t, Ts, Ts2, inv_l1);
              O[j] = row_terms(K, R.hhat, R.Lf, R.g0, R.g1, kLate ? at_o[j] : P.sigma_a * e_o[j], alpha_o[j]);
              acc_row(A, O[j]);
            }
          } else if (G * j < n_obs) {
            // lanes past the last obstacle read a staged blank obstacle (Q =
            // 0): its row has hhat = -1 and Lf = g = +-0, so it adds exact
            // zeros to the sums, without a divergent branch or selects
            const ObsRow R = obstacle_row_sel<E4, DISC>(sobs[o], DB, px, py, v, a, c1, s1, vkd, sec2, t, Ts, Ts2, inv_l1);
            O[j] = row_terms(K, R.hhat, R.Lf, R.g0, R.g1, kLate ? at_o[j] : P.sigma_a * e_o[j], alpha_o[j]);
            acc_row(A, O[j]);
          }
        }
        return A;
      };
      const Acc5 S8 = virtual_tree<G, 0, NV>(leaf);
      const double N00 = (double)Mj + S8.N00, N01 = S8.N01, N11 = (double)Mw + S8.N11;
      const double y0 = (double)(P.W_j * uj + pj0) + S8.y0;
      const double y1 = (double)(P.W_w * uw + pw0) + S8.y1;
      const double det = N00 * N11 - N01 * N01;
      // det > 0 (N is the diagonal W + rho I plus positive semidefinite rank-one
      // terms): the hardware reciprocal and one Newton step square its relative
      // error, far below the FP32 rounding of the result (3 instructions
      // instead of the IEEE division's 12)
      double idet = __builtin_amdgcn_rcp(det);
      idet = fma(fma(-det, idet, 1.0), idet, idet);
      uj = (float)((N11 * y0 - N01 * y1) * idet);
      uw = (float)((N00 * y1 - N01 * y0) * idet);
      // next barrier rates: alpha + u*alpha = -(Lf + g u*)/hh (eq. (9) holds exactly)
      if (G > 1 || hitch) {
#pragma unroll
        for (int k = 0; k < NH; ++k) alpha_h[k] = -(H[k].Lf + H[k].g0 * uj + H[k].g1 * uw) * H[k].ih;
      }
#pragma unroll
      for (int j = 0; j < NSL; ++j) {
        const int o = g + G * j;
        if (G == 1 ? (o < n_obs) : (G * j < n_obs)) alpha_o[j] = -(O[j].Lf + O[j].g0 * uj + O[j].g1 * uw) * O[j].ih;
      }
    }

    // --- stage cost r(x_tau, u*_tau, psi_tau), eq. (13) ---
    if constexpr (!kBatchCost) {
      float rc = stage_cost(P, rf, tg.sr, tg.cr, px, py, th1, th2, uj, uw, unu);
      if (penalty) rc += P.w_col * collision_pen<E4, DISC>(sobs, n_obs, px, py, th1, th2, t0 + (float)tau * Ts);
      J += (double)rc;
    } else {
      const bool mine = (int)(tau & (G - 1)) == g;
      k_px = sel(mine, px, k_px);
      k_py = sel(mine, py, k_py);
      k_th1 = sel(mine, th1, k_th1);
      k_th2 = sel(mine, th2, k_th2);
      k_psi = sel(mine, psi, k_psi);
      k_uj = sel(mine, uj, k_uj);
      k_uw = sel(mine, uw, k_uw);
      k_unu = sel(mine, unu, k_unu);
    }

    // --- applied inputs: [3T][S_pad] in HBM and/or the tile's LDS ---
    if (d.ustar_global && store) {
      stf<kGlb>(ustar + (size_t)(3 * tau + 0) * S_pad + s, uj);
      stf<kGlb>(ustar + (size_t)(3 * tau + 1) * S_pad + s, uw);
      stf<kGlb>(ustar + (size_t)(3 * tau + 2) * S_pad + s, unu);
    }
    if (s_u) {
      // every lane of the sample writes the same values to its column; the
      // column of a sample past S is never weighted
      s_u[(3 * tau + 0) * lds_stride + t_local] = uj;
      s_u[(3 * tau + 1) * lds_stride + t_local] = uw;
      s_u[(3 * tau + 2) * lds_stride + t_local] = unu;
    }

    // --- explicit Euler, eq. (6), plus psi_dot = nu ---
    const float npx = px + Ts * v * c1;
    const float npy = py + Ts * v * s1;
    const float nv = v + Ts * a;
    const float na = a + Ts * uj;
    const float nth1 = th1 + Ts * vkd;
    const float nth2 = th2 + Ts * v * inv_l2 * Aw2;
    const float ndl = dl + Ts * uw;
    psi = psi_next;
    px = npx;
    py = npy;
    v = nv;
    a = na;
    th1 = nth1;
    th2 = nth2;
    dl = ndl;
  };
  // costs of the kept steps tau0 .. tau0 + n - 1 (lane g: step tau0 + g)
  auto flush_costs = [&](uint32_t tau0, uint32_t n) __attribute__((always_inline)) {
    if constexpr (kBatchCost) {
      const RefPoint r = reference<kGlb, !kAhead>(phi0 + k_psi * inv_ds, k0, n_path, spath, w0, nw, gpath, ox, oy);
      float sr, cr;
      step_sincos(r.th1, &sr, &cr);
      float rc = stage_cost(P, r, sr, cr, k_px, k_py, k_th1, k_th2, k_uj, k_uw, k_unu);
      if (penalty)
        rc += P.w_col * collision_pen<E4, DISC>(sobs, n_obs, k_px, k_py, k_th1, k_th2,
                                                t0 + (float)(tau0 + (uint32_t)g) * Ts);
      J += (double)rc;
      if (n > 1) J += (double)lane_value<G, 1>(rc);
      if constexpr (G >= 4) {
        if (n > 2) J += (double)lane_value<G, 2>(rc);
        if (n > 3) J += (double)lane_value<G, 3>(rc);
      }
      if constexpr (G >= 8) {
        if (n > 4) J += (double)lane_value<G, 4>(rc);
        if (n > 5) J += (double)lane_value<G, 5>(rc);
        if (n > 6) J += (double)lane_value<G, 6>(rc);
        if (n > 7) J += (double)lane_value<G, 7>(rc);
      }
    }
  };
  auto after_step = [&](uint32_t tau) __attribute__((always_inline)) {
    if constexpr (kBatchCost) {
      if (((tau + 1) & (G - 1)) == 0 || tau + 1 == d.T) flush_costs(tau & ~(uint32_t)(G - 1), (tau & (G - 1)) + 1);
    }
  };
  if constexpr (kLate) {
    // whole pairs, then an odd last step: every pass of the loop issues both
    // slots' refills, so a step's wait for its own slot leaves the other
    // slot's loads in flight
    uint32_t tau = 0;
    for (; tau + 1 < d.T; tau += 2) {
      step(tau, std::integral_constant<int, 0>{});
      after_step(tau);
      step(tau + 1, std::integral_constant<int, 1>{});
      after_step(tau + 1);
    }
    if (tau < d.T) {
      step(tau, std::integral_constant<int, 0>{});
      after_step(tau);
    }
  } else if constexpr (PRE) {
    for (uint32_t tau = 0; tau < d.T; tau += 2) {
      step(tau, std::integral_constant<int, 0>{});
      after_step(tau);
      if (tau + 1 < d.T) {
        step(tau + 1, std::integral_constant<int, 1>{});
        after_step(tau + 1);
      }
    }
  } else {
    for (uint32_t tau = 0; tau < d.T; ++tau) step(tau, std::integral_constant<int, 0>{});
  }
  rf = reference<kGlb, !kAhead>(phi0 + psi * inv_ds, k0, n_path, spath, w0, nw, gpath, ox, oy);
  float rN = tracking_cost(P, rf, px, py, th1, th2);   // rf: the reference at psi_T
  if (penalty) rN += P.w_col * collision_pen<E4, DISC>(sobs, n_obs, px, py, th1, th2, t0 + (float)d.T * Ts);
  J += (double)rN;
  float Jf = (float)J;
  if (!isfinite(Jf)) Jf = INFINITY;
  if (store) {
    d.J[s] = Jf;
    if (s_J) s_J[t_local] = Jf;
  }
}


// ---------------------------------------------------------------------------
// Noise: every (four consecutive samples, step) in parallel, all their Philox
// blocks in one thread (independent chains the scheduler interleaves) ->
// [tau][k][S_pad], one 16-byte store per lane and row
// ---------------------------------------------------------------------------
constexpr int kMaxPhiloxBlocks = (5 + BRMPPI_MAX_OBS + 3) / 4;

__global__ __launch_bounds__(256) void k_noise(const char* __restrict__ descs, uint32_t stride, uint32_t nb) {
  // blockIdx.z = update u of a run of consecutive descriptors; a thread draws
  // four consecutive samples at step blockIdx.y and stores each row of normals
  // with one 16-byte store (samples from S up to S_pad get the normals of
  // their own indices, which nothing reads)
  const SolveDesc& d = *reinterpret_cast<const SolveDesc*>(descs + (size_t)blockIdx.z * stride);
  const uint32_t s0 = 4 * (blockIdx.x * blockDim.x + threadIdx.x);
  const uint32_t tau = blockIdx.y;
  if (s0 >= d.S_pad) return;
  float* __restrict__ out = d.noise + (size_t)tau * d.n_normals * d.S_pad + s0;
#pragma unroll
  for (int b = 0; b < kMaxPhiloxBlocks; ++b) {
    if ((uint32_t)b < nb) {
      float e[4][4];
#pragma unroll
      for (uint32_t i = 0; i < 4; ++i) {
        uint32_t r[4];
        philox4x32_10(s0 + i, tau, (uint32_t)b, d.instance, d.seed_lo, d.seed_hi, r);
        box_muller4(r, e[i]);
      }
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t kk = 4 * (uint32_t)b + k;
        if (kk < d.n_normals)
          gst4(reinterpret_cast<float4*>(out + (size_t)kk * d.S_pad), make_float4(e[0][k], e[1][k], e[2][k], e[3][k]));
      }
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

// Hand-off of partial results between blocks (the "last block" patterns).
// The partials are written and read only as device-scope relaxed atomics:
// such a store writes through its XCD's L2 and such a load does not take a
// stale line from the reader's L2, so each partial is coherent across the
// XCDs by itself.  A publisher then needs only every wave's stores complete
// (vmcnt drained) before the block's counter increment, and the block that
// sees the last increment reads with those loads after it.  A release fence
// at device scope would instead write back every dirty line of the XCD's L2
// (and an acquire invalidate it), which stalls every block on that XCD: one
// such write-back per work item cost the batched reduce a quarter of its
// time.
typedef __attribute__((address_space(1))) float glb_float;
__device__ __forceinline__ void pub_st(float* p, float v) {
  __hip_atomic_store((glb_float*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void pub_st4(float4* p, float4 v) {
  pub_st(&p->x, v.x);
  pub_st(&p->y, v.y);
  pub_st(&p->z, v.z);
  pub_st(&p->w, v.w);
}
__device__ __forceinline__ float pub_ld(const float* p) {
  return __hip_atomic_load((const glb_float*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float4 pub_ld4(const float4* p) {
  return make_float4(pub_ld(&p->x), pub_ld(&p->y), pub_ld(&p->z), pub_ld(&p->w));
}
// this wave's stores complete; also a compiler barrier, so that no store
// moves past it
__device__ __forceinline__ void pub_complete() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// the block's next work item.  Persistent launch (grid <= items): the first
// item of block b is item b, the later ones come from the queue, past the
// grid's first round (so that the whole grid does not start on one contended
// atomic).  Direct launch: item blockIdx.x only.
__device__ __forceinline__ bool next_item(uint32_t it, uint32_t n_items, uint32_t* ctr_next, uint32_t* s_slot,
                                          uint32_t& ix) {
  if (ctr_next) {
    if (it == 0) {
      ix = blockIdx.x;
    } else {
      if (threadIdx.x == 0) *s_slot = gridDim.x + atomicAdd(ctr_next, 1u);
      __syncthreads();
      ix = *s_slot;
    }
  } else {
    if (it > 0) return false;
    ix = blockIdx.x;
  }
  ix = __builtin_amdgcn_readfirstlane(ix);
  return ix < n_items;
}

// The last block to finish resets the queue for the next launch (a graph
// replay).  Only the two counters take part: a block increments done after
// its last grab of next has returned, so no fence is needed.
__device__ __forceinline__ void finish_persistent(uint32_t* next, uint32_t* done) {
  if (threadIdx.x == 0) {
    const uint32_t k = atomicAdd(done, 1u);
    if (k == gridDim.x - 1) {
      atomicExch(next, 0u);
      atomicExch(done, 0u);
    }
  }
}

// ---------------------------------------------------------------------------
// Weights, weighted reduction and update (Sec. III-B weights, eq. (5))
// ---------------------------------------------------------------------------
// The weights exp(-(J_s - m)/lambda) and the weighted average of the applied
// inputs are formed in a fixed structure so that the result never depends on
// the launch shape: a unit of 32 samples takes weights relative to its own
// minimum, a group of 32 units rescales them to the group minimum, and the
// last block of the instance rescales the groups to the global minimum
// (log-sum-exp merges) and writes U_new, the receding-horizon shift and, when
// asked, the closed-loop plant step.

// FP64 plant step of the closed loop (Sec. II model, inputs clipped to the
// hard bounds), in two halves so that only the last few operations wait for
// the merge.  s_plant: [0..5] sin/cos of th1, delta, th1 - th2; [6..13] the
// state; [14..16] the applied input U_new[0].
constexpr int kPlantLds = 17;
// first half (no barrier): lanes 0..7 load the state, lanes 0..2 one sincos each
__device__ __forceinline__ void plant_prep(const SolveDesc& d, double* s_plant) {
  const uint32_t t = threadIdx.x;
  const double* x = d.plant_x;
  if (t < 8) lds_put(s_plant + 6 + t, x[t]);
  if (t < 3) {
    const double ang = t == 0 ? x[4] : (t == 1 ? x[6] : x[4] - x[5]);
    double sn, cs;
    sincos(ang, &sn, &cs);
    lds_put(s_plant + 2 * t, sn);
    lds_put(s_plant + 2 * t + 1, cs);
  }
}
// Hitch-angle stabiliser (Sec. IV-D, eq. (19)) in FP64: (j, w) <- argmin of
// q_j (j - j_ref)^2 + q_w (w - w_ref)^2 over the input box subject to
// Lf + g u >= -alpha_h hhat for both hitch rows (the first-order expanded
// barrier of the rollouts).  The optimum of this strictly convex 2-D problem
// is the reference, the projection onto one constraint line, or a vertex of
// two: every candidate is formed and the feasible one with the least cost
// kept.  No feasible input: the reference clipped to the box.
__device__ bool hitch_qp(const brmppi_params& P, const double x[8], const double* s_plant, double& j, double& w) {
  const double Ts = P.Ts, l1 = P.l1, l2 = P.l2;
  const double v = x[2], a = x[3], phi = x[4] - x[5];
  const double sp = s_plant[4], cp = s_plant[5];
  const double tn = s_plant[2] / s_plant[3], sec2 = 1.0 + tn * tn;
  const double ch = (double)P.lh / l1, kd = tn / l1;
  const double Aw2 = sp - ch * cp * tn;
  const double D = v / l2 * Aw2 - v * kd;
  const double D_v = Aw2 / l2 - kd;
  const double D_phi = v / l2 * (cp + ch * sp * tn);
  const double D_dl = -v * sec2 * (ch * cp / l2 + 1.0 / l1);
  double A[6][2], c[6];
  for (int k = 0; k < 2; ++k) {
    const double sg = k == 0 ? 1.0 : -1.0;
    const double h = (double)P.dtheta_max - (double)P.kappa * v + sg * phi;
    const double hd = -(double)P.kappa * a - sg * D;
    const double hv = -(double)P.kappa - sg * Ts * D_v;
    const double Lf = Ts * (hv * a - sg * (1.0 - Ts * D_phi) * D);
    A[k][0] = -(double)P.kappa * Ts * Ts;
    A[k][1] = -sg * Ts * Ts * D_dl;
    c[k] = -(double)P.alpha_h * (h + Ts * hd) - Lf;
  }
  A[2][0] = 1.0;  A[2][1] = 0.0;  c[2] = P.j_lo;
  A[3][0] = -1.0; A[3][1] = 0.0;  c[3] = -(double)P.j_hi;
  A[4][0] = 0.0;  A[4][1] = 1.0;  c[4] = P.w_lo;
  A[5][0] = 0.0;  A[5][1] = -1.0; c[5] = -(double)P.w_hi;
  const double q0 = P.qh_j, q1 = P.qh_w;
  const double r0 = j, r1 = w;
  double best = INFINITY, b0 = 0.0, b1 = 0.0;
  auto consider = [&](double u0, double u1) {
    for (int i = 0; i < 6; ++i) {
      const double lhs = A[i][0] * u0 + A[i][1] * u1;
      const double scale = fabs(c[i]) + fabs(A[i][0] * u0) + fabs(A[i][1] * u1) + 1e-300;
      if (lhs - c[i] < -1e-10 * scale) return;
    }
    const double e0 = u0 - r0, e1 = u1 - r1;
    const double obj = q0 * e0 * e0 + q1 * e1 * e1;
    if (obj < best) {
      best = obj;
      b0 = u0;
      b1 = u1;
    }
  };
  consider(r0, r1);
  for (int i = 0; i < 6; ++i) {
    const double aQa = A[i][0] * A[i][0] / q0 + A[i][1] * A[i][1] / q1;
    if (!(aQa > 0.0)) continue;
    const double lam = (c[i] - (A[i][0] * r0 + A[i][1] * r1)) / aQa;
    consider(r0 + A[i][0] / q0 * lam, r1 + A[i][1] / q1 * lam);
  }
  for (int i = 0; i < 6; ++i) {
    for (int k = i + 1; k < 6; ++k) {
      const double det = A[i][0] * A[k][1] - A[i][1] * A[k][0];
      const double nrm = fabs(A[i][0] * A[k][1]) + fabs(A[i][1] * A[k][0]);
      if (!(fabs(det) > 1e-14 * nrm)) continue;
      consider((c[i] * A[k][1] - c[k] * A[i][1]) / det, (A[i][0] * c[k] - A[k][0] * c[i]) / det);
    }
  }
  if (!(best < INFINITY)) return false;
  j = b0;
  w = b1;
  return true;
}

// second half, one thread, after a barrier
__device__ __forceinline__ void plant_finish(const SolveDesc& d, const double* s_plant) {
  const brmppi_params& P = d.prm;
  double x[8];
  for (int k = 0; k < 8; ++k) x[k] = lds(s_plant + 6 + k);
  double j = lds(s_plant + 14), w = lds(s_plant + 15);
  const double nu = lds(s_plant + 16);
  const bool stabilised = (d.flags & BRMPPI_HITCH_QP) && hitch_qp(P, x, s_plant, j, w);
  if (!stabilised) {   // hard input bounds on the applied input
    j = fmin(fmax(j, (double)P.j_lo), (double)P.j_hi);
    w = fmin(fmax(w, (double)P.w_lo), (double)P.w_hi);
  }
  const double Ts = P.Ts, l1 = P.l1, l2 = P.l2, lh = P.lh;
  const double v = x[2], a = x[3];
  const double s1 = lds(s_plant + 0), c1 = lds(s_plant + 1);
  const double tan_dl = lds(s_plant + 2) / lds(s_plant + 3);
  const double s12 = lds(s_plant + 4), c12 = lds(s_plant + 5);
  double xn[8];
  xn[0] = x[0] + Ts * v * c1;
  xn[1] = x[1] + Ts * v * s1;
  xn[2] = v + Ts * a;
  xn[3] = a + Ts * j;
  xn[4] = x[4] + Ts * v / l1 * tan_dl;
  xn[5] = x[5] + Ts * v / l2 * (s12 - lh / l1 * c12 * tan_dl);
  xn[6] = x[6] + Ts * w;
  xn[7] = x[7] + Ts * nu;
  for (int k = 0; k < 8; ++k) d.plant_x[k] = xn[k];
}

// block-wide reductions in a fixed order (thread stride, wave butterfly, waves
// in index order): the same inputs give the same bits on every launch
__device__ __forceinline__ float block_min(float v, float* s_red) {
  v = wave_min(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds_put(s_red + (threadIdx.x >> 6), v);
  __syncthreads();
  float r = lds(s_red);
  for (uint32_t w = 1; w < blockDim.x / 64; ++w) r = fminf(r, lds(s_red + w));
  return r;
}
// two sums with one pair of barriers (s_red: 2 x 4 floats), each in the same
// order as a single block sum
__device__ __forceinline__ void block_sum2(float& a, float& b, float* s_red) {
  a = wave_sum(a);
  b = wave_sum(b);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    lds_put(s_red + (threadIdx.x >> 6), a);
    lds_put(s_red + 4 + (threadIdx.x >> 6), b);
  }
  __syncthreads();
  float ra = lds(s_red), rb = lds(s_red + 4);
  for (uint32_t w = 1; w < blockDim.x / 64; ++w) {
    ra += lds(s_red + w);
    rb += lds(s_red + 4 + w);
  }
  a = ra;
  b = rb;
}

// Merge of the group partials (a group = 1024 samples) by the last block of an
// instance: global min m = min_c m_c, group scale exp(-(m_c - m)/lambda), Z
// and sum of squared weights, then U = sum_c scale_c rpart[c] / Z per row
// (eq. (5)).  Every load is issued by a different thread or unrolled, so the
// merge costs a few memory latencies, not one per group.
__device__ void finalize_instance(const SolveDesc& d, float* s_scale, float* s_red, double* s_plant) {
  const uint32_t nW = d.n_wchunk;
  const uint32_t R = 3 * d.T;
  const uint32_t nt = blockDim.x;
  const bool plant = (d.flags & BRMPPI_ADVANCE_PLANT) != 0;
  if (plant) plant_prep(d, s_plant);   // overlaps the merge
  // the first 8 group partials of this thread's first row, loaded before the
  // merge's barriers so that their latency overlaps them
  constexpr int kPre = 8;
  const uint32_t r0 = threadIdx.x;
  float pre[kPre];
#pragma unroll
  for (int k = 0; k < kPre; ++k) pre[k] = (r0 < R && (uint32_t)k < nW) ? pub_ld(d.rpart + (size_t)k * R + r0) : 0.0f;
  // this thread's first group partial is loaded once, for the minimum and the sums
  const float4 w_first = threadIdx.x < nW ? pub_ld4(d.wpart + threadIdx.x) : make_float4(INFINITY, 0.0f, 0.0f, 0.0f);
  float mloc = w_first.x;
  for (uint32_t c = threadIdx.x + nt; c < nW; c += nt) {
    mloc = fminf(mloc, pub_ld(&d.wpart[c].x));
  }
  const float m = block_min(mloc, s_red);
  float zl = 0.0f, z2l = 0.0f;
  for (uint32_t c = threadIdx.x; c < nW; c += nt) {
    const float4 w = c == threadIdx.x ? w_first : pub_ld4(d.wpart + c);
    const float sc = (m < INFINITY && w.x < INFINITY) ? expf(-(w.x - m) * d.inv_lambda) : 0.0f;
    lds_put(s_scale + c, sc);
    zl += sc * w.y;
    z2l += sc * sc * w.z;
  }
  block_sum2(zl, z2l, s_red);   // also orders the s_scale stores before the reads below
  const float Z = zl, Z2 = z2l;
  const bool ok = (m < INFINITY) && (Z > 0.0f);
  if (ok) {
    const float iZ = 1.0f / Z;
    for (uint32_t r = threadIdx.x; r < R; r += nt) {
      const float* __restrict__ col = d.rpart + r;
      float acc = 0.0f;
      uint32_t c = 0;
      for (; c + kPre <= nW; c += kPre) {
        const bool use_pre = (c == 0) && (r == r0);
        float v[kPre];
#pragma unroll
        for (int k = 0; k < kPre; ++k) v[k] = use_pre ? pre[k] : pub_ld(col + (size_t)(c + k) * R);
#pragma unroll
        for (int k = 0; k < kPre; ++k) acc += lds(s_scale + c + k) * v[k];
      }
#pragma unroll
      for (int k = 0; k < kPre; ++k) {
        if (c + k < nW) {
          const float vk = (c == 0 && r == r0) ? pre[k] : pub_ld(col + (size_t)(c + k) * R);
          acc += lds(s_scale + c + k) * vk;
        }
      }
      const float U = acc * iZ;
      gst(d.u_new + r, U);
      if (plant && r < 3) lds_put(s_plant + 14 + r, (double)U);
      // receding-horizon shift: U_nom <- [U[1:], U[T-1]]
      if (r >= 3) gst(d.u_nom_out + r - 3, U);
      if (r + 3 >= R) gst(d.u_nom_out + r, U);
    }
  } else {
    // every cost non-finite: return the nominal sequence, keep the warm start
    for (uint32_t r = threadIdx.x; r < R; r += nt) {
      const float U = gld(d.u_nom_in + r);
      gst(d.u_new + r, U);
      if (plant && r < 3) lds_put(s_plant + 14 + r, (double)U);
    }
  }
  if (threadIdx.x == 0) {
    d.stats[0] = m;
    d.stats[1] = Z;
    d.stats[2] = ok ? Z * Z / Z2 : 0.0f;
    d.stats[3] = ok ? (float)BRMPPI_OK : (float)BRMPPI_ENONFINITE;
  }
  if (plant) {
    __syncthreads();                 // U_new[0] from threads 0..2, the state and sines
    if (threadIdx.x == 0) plant_finish(d, s_plant);
  }
}

// ---------------------------------------------------------------------------
// Canonical reduction primitives (Sec. III-B weights and eq. (5)).  The fused
// rollout epilogue and k_reduce both call exactly these, so a unit's or a
// group's partial has the same bits whichever kernel computes it.
// ---------------------------------------------------------------------------
// weight of a sample relative to its unit's minimum m (0 for non-finite costs
// and samples past S, which carry J = +inf)
__device__ __forceinline__ float unit_weight(float j, float m, float inv_lambda) {
  return (m < INFINITY && j < INFINITY) ? expf(-(j - m) * inv_lambda) : 0.0f;
}
// Z_u and the sum of squared weights over the unit's samples, in sample order
__device__ __forceinline__ void unit_sums(const float* gam, float& z, float& z2) {
  z = 0.0f;
  z2 = 0.0f;
#pragma unroll
  for (int i = 0; i < kUnit; ++i) {
    const float gm = lds(gam + i);
    z = z + gm;
    z2 = fmaf(gm, gm, z2);
  }
}
// one term of a unit's row sum: zero weights leave the sum as it is (samples
// past S hold no data)
__device__ __forceinline__ float unit_row_term(float acc, float gm, float u) {
  return gm != 0.0f ? fmaf(gm, u, acc) : acc;
}
// scale of a unit (or group) with minimum m inside a merge with minimum mg
__device__ __forceinline__ float merge_scale(float m, float mg, float inv_lambda) {
  return (mg < INFINITY && m < INFINITY) ? expf(-(m - mg) * inv_lambda) : 0.0f;
}
// group (Z, Z2) from its units' (m_u, Z_u, Z2_u) and scales, in unit order
// (entries are read kChunk at a time, in bounds, before any of them is used,
// so that the reads are not serialised behind the per-unit condition)
constexpr int kChunk = 8;
__device__ __forceinline__ void group_sums(const float4* up, const float* sig, uint32_t nu, float& z, float& z2) {
  z = 0.0f;
  z2 = 0.0f;
#pragma unroll
  for (int c = 0; c < kGroupUnits; c += kChunk) {
    float sc[kChunk];
    float4 q[kChunk];
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      q[k] = lds(up + c + k);
      sc[k] = lds(sig + c + k);
    }
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      if ((uint32_t)(c + k) < nu) {
        z = fmaf(sc[k], q[k].y, z);
        z2 = fmaf(sc[k] * sc[k], q[k].z, z2);
      }
    }
  }
}

// Group merge by the last tile of the group: m_g, unit scales, (Z_g, Z2_g)
// and the group row sums from the units' partials.
__device__ __forceinline__ void group_merge(const SolveDesc& d, uint32_t grp, uint32_t gu0, uint32_t nu_g, float* s_sig,
                            float4* s_up, float* s_red) {
  const uint32_t t = threadIdx.x, nt = blockDim.x, R = 3 * d.T;
  // this thread's first row: all the group's unit sums, loaded before the
  // minimum (they do not depend on it)
  // (units past nu_g read the group's last unit, in range; only terms of units
  // below nu_g are ever used)
  float v0[kGroupUnits];
  {
    const float* __restrict__ col = d.urow + (size_t)gu0 * R + (t < R ? t : 0);
#pragma unroll
    for (int u = 0; u < kGroupUnits; ++u) v0[u] = pub_ld(col + (size_t)min((uint32_t)u, nu_g - 1) * R);
  }
  float4 up = make_float4(INFINITY, 0.0f, 0.0f, 0.0f);
  if (t < nu_g) up = pub_ld4(d.upart + gu0 + t);
  const float mg = block_min(up.x, s_red);
  if (t < nu_g) {
    lds_put(s_up + t, up);
    lds_put(s_sig + t, merge_scale(up.x, mg, d.inv_lambda));
  }
  __syncthreads();
  // the group's (Z, Z2), on the first thread of a wave without a row when there
  // is one, so that it overlaps the row sums instead of preceding them
  const uint32_t tz = ((R + 63u) & ~63u) < nt ? ((R + 63u) & ~63u) : 0u;
  if (t == tz) {
    float z, z2;
    group_sums(s_up, s_sig, nu_g, z, z2);
    pub_st4(d.wpart + grp, make_float4(mg, z, z2, 0.0f));
  }
  // one row: its unit sums in v, the scales read kChunk at a time (in bounds,
  // before any of them is used)
  auto row_sum = [&](uint32_t r, const float* v) __attribute__((always_inline)) {
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < kGroupUnits; c += kChunk) {
      float sg[kChunk];
#pragma unroll
      for (int k = 0; k < kChunk; ++k) sg[k] = lds(s_sig + c + k);
#pragma unroll
      for (int k = 0; k < kChunk; ++k)
        if ((uint32_t)(c + k) < nu_g) acc = unit_row_term(acc, sg[k], v[c + k]);
    }
    pub_st(d.rpart + (size_t)grp * R + r, acc);
  };
  if (t < R) row_sum(t, v0);
  for (uint32_t r = t + nt; r < R; r += nt) {
    // all the group's unit sums of this row are loaded at once: one latency
    const float* __restrict__ col = d.urow + (size_t)gu0 * R + r;
    float v[kGroupUnits];
#pragma unroll
    for (int u = 0; u < kGroupUnits; ++u) v[u] = pub_ld(col + (size_t)min((uint32_t)u, nu_g - 1) * R);
    row_sum(r, v);
  }
}

// Fused reduction of one tile (its samples' costs and applied inputs are in
// LDS): unit weights, unit partials to HBM; the last tile of each group merges
// the group, the last group the instance (U_new, shift, plant step).
// Waves per SIMD the register allocation must leave room for.  Up to 16
// obstacle slots every launch shape fits two waves (the one-lane forms with a
// few spilled values, which still pays: at one wave per SIMD nothing hides the
// step's latency), and so do the four- and eight-lane forms with 32 slots (a
// lane holds 8 or 4 obstacle rows); the one- and two-lane forms with 32 slots
// would spill hundreds of values, so they keep the whole register file.
template <int NOB, int G>
constexpr int rollout_waves_per_simd() {
  return (NOB <= 16 || G >= 4) ? 2 : 1;
}

// Inlined into the kernel: as a function call, every lane saved and restored
// its callee-saved registers around it (tens of bytes of scratch per lane).
__device__ __forceinline__ void tile_epilogue(const SolveDesc& d, uint32_t s0, uint32_t per_tile, float* s_u, uint32_t lds_stride,
                              const float* s_J, float* s_gam, float* s_mu, float* s_sig, float4* s_up,
                              float* s_red, double* s_trig, uint32_t* s_flag) {
  const uint32_t t = threadIdx.x, nt = blockDim.x, R = 3 * d.T;
  const uint32_t k_units = per_tile / kUnit;
  const uint32_t u0 = s0 / kUnit;
  const uint32_t nu_tile = min(k_units, d.n_units - u0);
  // unit minimum (exact in any order) and weights; a unit is half a wave
  if (t < per_tile) {
    const float j = lds(s_J + t);
    float m = j;
#pragma unroll
    for (int o = kUnit / 2; o >= 1; o >>= 1) m = fminf(m, __shfl_xor(m, o, 64));
    lds_put(s_gam + t, unit_weight(j, m, d.inv_lambda));
    if ((t & (kUnit - 1)) == 0) lds_put(s_mu + t / kUnit, m);
  }
  __syncthreads();
  if (t < nu_tile) {
    float z, z2;
    unit_sums(s_gam + kUnit * t, z, z2);
    pub_st4(d.upart + u0 + t, make_float4(lds(s_mu + t), z, z2, 0.0f));
  }
  for (uint32_t it = t; it < nu_tile * R; it += nt) {
    const uint32_t j = it / R, r = it - j * R;
    const float* gam = s_gam + kUnit * j;
    const float* u = s_u + r * lds_stride + kUnit * j;
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < kUnit; c += kChunk) {
      float g8[kChunk], u8[kChunk];
#pragma unroll
      for (int k = 0; k < kChunk; ++k) {
        g8[k] = lds(gam + c + k);
        u8[k] = lds(u + c + k);
      }
#pragma unroll
      for (int k = 0; k < kChunk; ++k) acc = unit_row_term(acc, g8[k], u8[k]);
    }
    pub_st(d.urow + (size_t)(u0 + j) * R + r, acc);
  }
  // publish the tile's units; the last tile of the group merges it
  const uint32_t grp = u0 / kGroupUnits, gu0 = grp * kGroupUnits;
  const uint32_t nu_g = min((uint32_t)kGroupUnits, d.n_units - gu0);
  const uint32_t tiles_g = (nu_g + k_units - 1) / k_units;
  pub_complete();
  __syncthreads();
  if (t == 0) *s_flag = (atomicAdd(&d.gctr[grp * kCtrStride], 1u) == tiles_g - 1) ? 1u : 0u;
  __syncthreads();
  if (*s_flag == 0u) return;
  group_merge(d, grp, gu0, nu_g, s_sig, s_up, s_red);
  if (t == 0) atomicExch(&d.gctr[grp * kCtrStride], 0u);
  // publish the group; the last group merges the instance
  pub_complete();
  __syncthreads();
  if (t == 0) *s_flag = (atomicAdd(d.counter, 1u) == d.n_wchunk - 1) ? 1u : 0u;
  __syncthreads();
  if (*s_flag == 0u) return;
  finalize_instance(d, s_u, s_red, s_trig);   // the inputs' LDS is free: merge scales
  if (t == 0) atomicExch(d.counter, 0u);
}

template <int NOB, bool GUIDED, int G, bool PRE>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(rollout_waves_per_simd<NOB, G>(), 8)))
void k_rollout(const SolveDesc* __restrict__ descs,
                                                       const Tile* __restrict__ tiles, uint32_t n_tiles,
                                                       BatchCounters* __restrict__ ctr) {
  __shared__ float4 s_path[kPathWin];
  __shared__ float s_unom[3 * BRMPPI_MAX_T];
  __shared__ ObsL s_obs[BRMPPI_MAX_OBS];
  __shared__ uint32_t s_tile, s_flag;
  __shared__ float s_red[2 * (kMaxBlock / 64)];
  __shared__ double s_trig[kPlantLds];
  extern __shared__ float s_dyn[];            // fused epilogue only
  const uint32_t per_tile = blockDim.x / G;   // samples per tile
  const uint32_t lds_stride = per_tile + 1;
  for (uint32_t it = 0;; ++it) {
    uint32_t tix;
    if (!next_item(it, n_tiles, ctr ? &ctr->tile_next : nullptr, &s_tile, tix)) break;
    Tile tl;
    if (tiles) {
      tl = tiles[tix];
    } else {
      tl.inst = 0;
      tl.s0 = tix * per_tile;
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

    // stage the obstacle rows (row r: obstacle r % n_objects around footprint
    // disc r / n_objects) and the path window
    if (threadIdx.x < d.n_obs) {
      const uint32_t oi = threadIdx.x % d.n_objects;
      const brmppi_obstacle o = d.obs[oi];
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
      L.e4 = (o.e == 4.0f) ? 1.0f : 0.0f;
      L.co = co;
      L.so = so;
      L.k0 = (o.e == 4.0f) ? iax * iax : iax;   // (m + r)^-e
      L.k1 = (o.e == 4.0f) ? iay * iay : iay;
      disc_ab(d.prm, threadIdx.x / d.n_objects, L.dA, L.dB);
      s_obs[threadIdx.x] = L;
    } else if (threadIdx.x < BRMPPI_MAX_OBS) {
      // blank slots (Q = 0, k = 0, at rest): the rows of lanes past the last
      // obstacle row
      s_obs[threadIdx.x] = ObsL{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    }
    // the path window and (forms with fewer than eight lanes) the nominal
    // inputs, 3T floats, their first loads all issued before the first store
    // (the window's 4 per thread at 256 threads): one memory latency, not
    // one per value a thread stages
    const int R3 = 3 * (int)d.T, bd = (int)blockDim.x, tx = (int)threadIdx.x;
    float un0 = 0.0f, un1 = 0.0f;
    if constexpr (G < 8) {
      un0 = gld(d.u_nom_in + min(tx, R3 - 1));
      un1 = gld(d.u_nom_in + min(tx + bd, R3 - 1));
    }
    for (int j0 = 0; j0 < nw; j0 += 4 * (int)blockDim.x) {
      float4 w[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) w[k] = d.path[w0 + min(j0 + k * (int)blockDim.x + (int)threadIdx.x, nw - 1)];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int j = j0 + k * (int)blockDim.x + (int)threadIdx.x;
        if (j < nw) s_path[j] = make_float4(w[k].x - ox, w[k].y - oy, w[k].z, w[k].w);
      }
    }
    if constexpr (G < 8) {
      if (tx < R3) s_unom[tx] = un0;
      if (tx + bd < R3) s_unom[tx + bd] = un1;
      for (int r = tx + 2 * bd; r < R3; r += bd) s_unom[r] = gld(d.u_nom_in + r);
    }
    // fused epilogue (direct launch of one instance): LDS for the tile's
    // applied inputs, costs (+inf where no sample stores), weights, units
    const bool fused = (ctr == nullptr) && d.fused;
    float *s_u = nullptr, *s_J = nullptr, *s_gam = nullptr, *s_mu = nullptr, *s_sig = nullptr;
    float4* s_up = nullptr;
    if (fused) {
      s_u = s_dyn;
      s_J = s_dyn + fused_lds_region(per_tile, d.T, d.n_wchunk);
      s_gam = s_J + per_tile;
      s_mu = s_gam + per_tile;
      s_sig = s_mu + kGroupUnits;
      s_up = reinterpret_cast<float4*>(s_sig + kGroupUnits);
      for (uint32_t i = threadIdx.x; i < per_tile; i += blockDim.x) s_J[i] = INFINITY;
    }
    __syncthreads();

    // every lane runs (lanes past S repeat the last sample and do not store),
    // so the group-wide DPP broadcasts always read active lanes
    const uint32_t t_local = threadIdx.x / G;
    const uint32_t s_raw = tl.s0 + t_local;
    const int g = (int)(threadIdx.x % G);
    const bool valid = s_raw < d.S;
    const uint32_t s = valid ? s_raw : d.S - 1;
    bool done = false;
    if constexpr (GUIDED) {
      if (d.any_disc) {
        rollout_sample<NOB, GUIDED, G, PRE, true, true>(d, s, valid && g == 0, g, x0, s_obs, s_path, s_unom, w0, nw, k0,
                                                        phi0, s_u, lds_stride, t_local, s_J);
        done = true;
      }
    }
    if (!done) {
      if (d.any_e4)
        rollout_sample<NOB, GUIDED, G, PRE, true, false>(d, s, valid && g == 0, g, x0, s_obs, s_path, s_unom, w0, nw, k0,
                                                         phi0, s_u, lds_stride, t_local, s_J);
      else
        rollout_sample<NOB, GUIDED, G, PRE, false, false>(d, s, valid && g == 0, g, x0, s_obs, s_path, s_unom, w0, nw, k0,
                                                          phi0, s_u, lds_stride, t_local, s_J);
    }
    __syncthreads();
    if (fused)
      tile_epilogue(d, tl.s0, per_tile, s_u, lds_stride, s_J, s_gam, s_mu, s_sig, s_up, s_red, s_trig, &s_flag);
  }
  if (ctr) finish_persistent(&ctr->tile_next, &ctr->tile_done);
}

constexpr uint32_t kMaxWChunks = BRMPPI_MAX_S / kWChunk;
static_assert(kRowsPerPass == 2 * (kWThreads / 64), "two rows per wave and pass");
static_assert(kMaxRowsPerItem % kRowsPerPass == 0 && kMaxRowsPerItem <= kWThreads, "whole passes");
static_assert(kWChunk == 4 * kWThreads, "four samples per thread");
static_assert(kUnit == 32 && kGroupUnits == 32, "a unit is half a wave; a group's units fit one wave");

// Reduction from the applied inputs in HBM (batched launches and tiles that
// are not whole units), with the same canonical structure as the fused
// epilogue.  Work item = (group of 1024 samples, d.rows_item rows, up to
// 256): the group's unit weights are recomputed from its 4 KB of costs (same
// code: same values), the first row block also stores the group's (m_g, Z_g,
// Z2_g).  Wave w owns the group's samples 256 w .. 256 w + 255 (units 8 w ..
// 8 w + 7) and takes the item's rows 8 at a time: each row is read with one
// coalesced 16-byte load per lane, the 8 rows go through a padded LDS tile of
// the wave, and lane l then sums unit l % 8 of row l / 8 over its 32 samples
// in sample order (the weights of its unit are held in registers).  The next
// two passes' loads are in flight meanwhile.  The unit sums go to LDS and are
// merged in unit order by one thread per row; the item is published once.
// The last block of the instance merges the groups, with the group scales in
// the tiles' LDS.  Two blocks share a CU (LDS).
constexpr int kRedRows = 8;                          // rows per wave and pass
constexpr int kRedUnitStride = kUnit + 4;            // floats per unit segment in the tile (16 B pad)
constexpr int kRedRowStride = 8 * kRedUnitStride;    // floats per row of a wave's tile
static_assert(kRedRows * 8 == 64, "one (row, unit) pair per lane");

__global__ __launch_bounds__(kWThreads) void k_reduce(const SolveDesc* __restrict__ descs,
                                                     const Item* __restrict__ items, uint32_t n_items,
                                                     BatchCounters* __restrict__ ctr) {
  __shared__ float4 s_gam4[kWChunk / 4];
  __shared__ float s_mu[kGroupUnits], s_sig[kGroupUnits];
  __shared__ float4 s_up[kGroupUnits];
  __shared__ float s_R[kMaxRowsPerItem][kGroupUnits + 1];   // +1: row-wise reads hit distinct banks
  __shared__ float4 s_T4[(kWThreads / 64) * kRedRows * kRedRowStride / 4];
  __shared__ float s_red[2 * (kWThreads / 64)];
  __shared__ double s_trig[kPlantLds];
  __shared__ uint32_t s_slot, s_last;
  const uint32_t t = threadIdx.x;
  const int lane = t & 63, wid = t >> 6;
  const float* s_gam = reinterpret_cast<const float*>(s_gam4);
  float* s_T = reinterpret_cast<float*>(s_T4) + wid * (kRedRows * kRedRowStride);
  // the instance merge's group scales use the tiles' LDS (free by then)
  float* s_scale = reinterpret_cast<float*>(s_T4);
  static_assert(sizeof(s_T4) >= kMaxWChunks * sizeof(float), "group scales fit the tiles");
  // this lane's place in the wave's tile when storing (sample 4 lane of each
  // row) and when summing (unit lu of row lr)
  const uint32_t st_off = (uint32_t)(lane >> 3) * kRedUnitStride + 4 * (uint32_t)(lane & 7);
  const uint32_t lu = (uint32_t)lane & 7u, lr = (uint32_t)lane >> 3;
  for (uint32_t it = 0;; ++it) {
    uint32_t ix;
    if (!next_item(it, n_items, ctr ? &ctr->r_next : nullptr, &s_slot, ix)) break;
    Item item;
    if (items) {
      item = items[ix];
    } else {
      item.inst = 0;
      item.idx = ix;
    }
    const SolveDesc& d = descs[__builtin_amdgcn_readfirstlane(item.inst)];
    const uint32_t grp = item.idx / d.n_rgroup, rg = item.idx % d.n_rgroup;
    const uint32_t base = grp * kWChunk;
    const uint32_t R = 3 * d.T;
    const uint32_t S = d.S;
    const uint32_t gu0 = grp * kGroupUnits;
    const uint32_t nu_g = min((uint32_t)kGroupUnits, d.n_units - gu0);
    const uint32_t r0 = rg * d.rows_item;
    const uint32_t nrow = min(d.rows_item, R - r0);

    // thread t: samples 4t .. 4t + 3 of the group (unit t / 8); S_pad is a
    // multiple of 256, so a wave's samples are all inside the buffer or none.
    // Every load below is unconditional (a wave past S_pad reads the row's
    // last 16 bytes and gets weight 0), so that a wait for one pass's rows
    // can leave the next pass's loads in flight.
    const uint32_t s4 = base + 4 * t;
    const bool sv = s4 < d.S_pad;
    const uint32_t s4c = sv ? s4 : d.S_pad - 4;
    const float* __restrict__ colp = d.u_star + s4c;
    // the costs first: waiting for them does not wait for the rows
    const float4 jc = gld4(reinterpret_cast<const float4*>(d.J + s4c));
    // two passes of 8 rows in flight: pass p (p / 8 even) in slot 0, the next
    // in slot 1; a slot is refilled with the pass 16 rows on as soon as its
    // rows are in the tile.  Rows past nrow repeat the item's last row (cache
    // hits; their sums are not stored): with no branch around a load, the
    // wait for one slot never drains the other.
    float4 q[2][kRedRows];
    auto load_rows = [&](uint32_t p, auto SLOT) __attribute__((always_inline)) {
      constexpr int sl = decltype(SLOT)::value;
#pragma unroll
      for (int j = 0; j < kRedRows; ++j) {
        const uint32_t rr = min(p + (uint32_t)j, nrow - 1);
        // global-space loads: a flat load would also count against the LDS wait
        // counter, and the tile's LDS reads would wait for the next rows' loads
        q[sl][j] = gld4(reinterpret_cast<const float4*>(colp + (size_t)(r0 + rr) * d.S_pad));
      }
    };
    using Slot0 = std::integral_constant<int, 0>;
    using Slot1 = std::integral_constant<int, 1>;
    load_rows(0u, Slot0{});    // in flight while the weights are formed
    load_rows((uint32_t)kRedRows, Slot1{});

    // costs and unit weights
    float jv[4] = {jc.x, jc.y, jc.z, jc.w};
    float m = INFINITY;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (!(s4 + k < S) || !(jv[k] < INFINITY)) jv[k] = INFINITY;  // past S (or S_pad) or NaN -> weight 0
      m = fminf(m, jv[k]);
    }
    m = fminf(m, __shfl_xor(m, 1, 64));
    m = fminf(m, __shfl_xor(m, 2, 64));
    m = fminf(m, __shfl_xor(m, 4, 64));
    s_gam4[t] = make_float4(unit_weight(jv[0], m, d.inv_lambda), unit_weight(jv[1], m, d.inv_lambda),
                            unit_weight(jv[2], m, d.inv_lambda), unit_weight(jv[3], m, d.inv_lambda));
    if ((t & 7) == 0) s_mu[t >> 3] = m;
    __syncthreads();
    // group minimum and unit scales
    if (wid == 0) {
      float mg = (lane < (int)nu_g) ? s_mu[lane] : INFINITY;
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) mg = fminf(mg, __shfl_xor(mg, o, 64));
      if (lane < (int)nu_g) {
        s_sig[lane] = merge_scale(s_mu[lane], mg, d.inv_lambda);
        if (rg == 0) {
          float z, z2;
          unit_sums(s_gam + kUnit * lane, z, z2);
          s_up[lane] = make_float4(s_mu[lane], z, z2, 0.0f);
        }
      }
      if (lane == 0) s_red[0] = mg;
    }
    // the weights of the unit this lane sums
    float gw[kUnit];
    {
      const float4* g4 = s_gam4 + (kUnit / 4) * (8 * (uint32_t)wid + lu);
#pragma unroll
      for (int k = 0; k < kUnit / 4; ++k) {
        const float4 w = g4[k];
        gw[4 * k + 0] = w.x;
        gw[4 * k + 1] = w.y;
        gw[4 * k + 2] = w.z;
        gw[4 * k + 3] = w.w;
      }
    }
    // unit row sums, in sample order, 8 rows per pass
    auto pass = [&](uint32_t p, auto SLOT) __attribute__((always_inline)) {
      constexpr int sl = decltype(SLOT)::value;
#pragma unroll
      for (int j = 0; j < kRedRows; ++j)
        *reinterpret_cast<float4*>(s_T + j * kRedRowStride + st_off) = q[sl][j];
      load_rows(p + 2 * kRedRows, SLOT);
      __builtin_amdgcn_wave_barrier();
      const float4* u4 = reinterpret_cast<const float4*>(s_T + lr * kRedRowStride + lu * kRedUnitStride);
      float acc = 0.0f;
#pragma unroll
      for (int k = 0; k < kUnit / 4; ++k) {
        const float4 u = u4[k];
        acc = unit_row_term(acc, gw[4 * k + 0], u.x);
        acc = unit_row_term(acc, gw[4 * k + 1], u.y);
        acc = unit_row_term(acc, gw[4 * k + 2], u.z);
        acc = unit_row_term(acc, gw[4 * k + 3], u.w);
      }
      if (p + lr < nrow) s_R[p + lr][8 * wid + lu] = acc;
      __builtin_amdgcn_wave_barrier();
    };
    for (uint32_t p = 0; p < nrow; p += 2 * kRedRows) {
      pass(p, Slot0{});
      pass(p + kRedRows, Slot1{});
    }
    __syncthreads();
    if (rg == 0 && t == kWThreads - 1) {   // a thread without a row: overlaps the row merges
      float z, z2;
      group_sums(s_up, s_sig, nu_g, z, z2);
      pub_st4(d.wpart + grp, make_float4(s_red[0], z, z2, 0.0f));
    }
    // group row sums, in unit order
    if (t < nrow) {
      float acc = 0.0f;
      for (uint32_t v = 0; v < nu_g; ++v) acc = unit_row_term(acc, s_sig[v], s_R[t][v]);
      pub_st(d.rpart + (size_t)grp * R + r0 + t, acc);
    }
    // publish: the barrier completes every wave's stores, one release by
    // thread 0 then makes them visible to the block that finishes the instance
    pub_complete();
    __syncthreads();
    if (t == 0) {
      const uint32_t k = atomicAdd(d.counter, 1u);
      s_last = (k == d.n_ritems - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (s_last) {
      finalize_instance(d, s_scale, s_red, s_trig);
      if (t == 0) atomicExch(d.counter, 0u);
    }
    __syncthreads();
  }
  if (ctr) finish_persistent(&ctr->r_next, &ctr->r_done);
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

// the radius and the two angle factors of box_muller4 for raw words r
__global__ void k_box_muller_dump(const uint32_t* __restrict__ r, uint32_t n, float* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float u = unif23(r[i]);
  out[3 * (size_t)i] = bm_radius(u);
  out[3 * (size_t)i + 1] = __builtin_amdgcn_cosf(u);
  out[3 * (size_t)i + 2] = __builtin_amdgcn_sinf(u);
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// rollout variants: 0 = one lane per sample, in-kernel noise; 1 = one lane,
// precomputed noise; 2 / 3 / 4 = two / four / eight lanes per sample,
// precomputed noise
int variant_lanes(int variant) { return variant == 2 ? 2 : (variant == 3 ? 4 : (variant == 4 ? 8 : 1)); }
bool variant_pre(int variant) { return variant != 0; }

template <int NOB, bool GD, int G, bool PRE>
static hipError_t launch_rollout_t(const SolveDesc* descs, const Tile* tiles, uint32_t n_tiles,
                                   BatchCounters* ctr, uint32_t grid, uint32_t block, size_t lds,
                                   hipStream_t stream) {
  hipLaunchKernelGGL((k_rollout<NOB, GD, G, PRE>), dim3(grid), dim3(block), lds, stream, descs, tiles, n_tiles, ctr);
  return hipGetLastError();
}

template <int NOB, bool GD>
static hipError_t launch_variant(int variant, const SolveDesc* descs, const Tile* tiles, uint32_t n_tiles,
                                 BatchCounters* ctr, uint32_t grid, uint32_t block, size_t lds, hipStream_t stream) {
  switch (variant) {
    case 0: return launch_rollout_t<NOB, GD, 1, false>(descs, tiles, n_tiles, ctr, grid, block, lds, stream);
    case 1: return launch_rollout_t<NOB, GD, 1, true>(descs, tiles, n_tiles, ctr, grid, block, lds, stream);
    case 2:
      if constexpr (GD) return launch_rollout_t<NOB, GD, 2, true>(descs, tiles, n_tiles, ctr, grid, block, lds, stream);
      return hipErrorInvalidValue;
    case 3:
      if constexpr (GD) return launch_rollout_t<NOB, GD, 4, true>(descs, tiles, n_tiles, ctr, grid, block, lds, stream);
      return hipErrorInvalidValue;
    case 4:
      if constexpr (GD) return launch_rollout_t<NOB, GD, 8, true>(descs, tiles, n_tiles, ctr, grid, block, lds, stream);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rollout(int bucket, int variant, const SolveDesc* descs, const Tile* tiles, uint32_t n_tiles,
                          BatchCounters* ctr, uint32_t grid, uint32_t block, size_t lds, hipStream_t stream) {
  if (block == 0 || block > (uint32_t)kMaxBlock || (block % 64) != 0) return hipErrorInvalidValue;
  switch (bucket) {
    case 0: return launch_variant<0, false>(variant, descs, tiles, n_tiles, ctr, grid, block, lds, stream);
    case 2: return launch_variant<2, true>(variant, descs, tiles, n_tiles, ctr, grid, block, lds, stream);
    case 8: return launch_variant<8, true>(variant, descs, tiles, n_tiles, ctr, grid, block, lds, stream);
    case 16: return launch_variant<16, true>(variant, descs, tiles, n_tiles, ctr, grid, block, lds, stream);
    case 32: return launch_variant<32, true>(variant, descs, tiles, n_tiles, ctr, grid, block, lds, stream);
    default: return hipErrorInvalidValue;
  }
}

template <int NOB, bool GD, int G, bool PRE>
static int occ_t(uint32_t block) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rollout<NOB, GD, G, PRE>, (int)block, 0) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

template <int NOB, bool GD>
static int occ_variant(int variant, uint32_t block) {
  switch (variant) {
    case 1: return occ_t<NOB, GD, 1, true>(block);
    case 2:
      if constexpr (GD) return occ_t<NOB, GD, 2, true>(block);
      return 1;
    case 3:
      if constexpr (GD) return occ_t<NOB, GD, 4, true>(block);
      return 1;
    case 4:
      if constexpr (GD) return occ_t<NOB, GD, 8, true>(block);
      return 1;
    default: return occ_t<NOB, GD, 1, false>(block);
  }
}

int rollout_blocks_per_cu(int bucket, int variant, uint32_t block) {
  switch (bucket) {
    case 0: return occ_variant<0, false>(variant, block);
    case 2: return occ_variant<2, true>(variant, block);
    case 8: return occ_variant<8, true>(variant, block);
    case 16: return occ_variant<16, true>(variant, block);
    default: return occ_variant<32, true>(variant, block);
  }
}

hipError_t launch_noise(const SolveDesc* first, size_t stride, uint32_t count, uint32_t S, uint32_t T,
                        uint32_t n_normals, hipStream_t stream) {
  const uint32_t nb = (n_normals + 3) / 4;
  if (count == 0 || nb == 0 || nb > (uint32_t)kMaxPhiloxBlocks) return count == 0 || nb == 0 ? hipSuccess : hipErrorInvalidValue;
  const uint32_t S_pad = (S + 255u) & ~255u;   // the noise buffer's row length
  const dim3 grid((S_pad + 1023) / 1024, T, count);
  hipLaunchKernelGGL(k_noise, grid, dim3(256), 0, stream, reinterpret_cast<const char*>(first), (uint32_t)stride, nb);
  return hipGetLastError();
}


hipError_t launch_reduce(const SolveDesc* descs, const Item* items, uint32_t n_items, BatchCounters* ctr,
                         uint32_t grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_reduce, dim3(grid), dim3(kWThreads), 0, stream, descs, items, n_items, ctr);
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

hipError_t launch_box_muller_dump(const uint32_t* r, uint32_t n, float* out, hipStream_t stream) {
  const uint32_t b = 256, g = (n + b - 1) / b;
  if (g == 0) return hipSuccess;
  hipLaunchKernelGGL(k_box_muller_dump, dim3(g), dim3(b), 0, stream, r, n, out);
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
