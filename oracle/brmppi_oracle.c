/*
 * FP64 CPU oracle for one BR-MPPI control update -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct C.  Only tests/, __graft_entry__.smoke() and
 * bench.py's cpu_baseline leg may load or call it; the HIP library never does.
 *
 * Paper: "GPU-Accelerated Barrier-Rate Guided MPPI Control for Tractor-Trailer
 * Systems" (arXiv 2508.05773).  Section / equation numbers below are the
 * paper's.  Readings where the paper is silent or ambiguous are marked READING.
 *
 * Pins (tests/test_oracle_*.py): Philox bit-exact against an independent
 * big-integer implementation and against rocRAND; Box-Muller identity and a KS
 * test; closed-form straight-line, constant-curvature and trailer fixed-point
 * trajectories; barrier gradients by central differences and by a symbolic
 * (sympy) derivation; projection KKT conditions, textbook special cases and an
 * independent elimination; contouring error geometry; weight identities and
 * limits; and an end-to-end 50-digit mpmath re-derivation at S = 4, T = 3.
 */
#include "brmppi_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Noise: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) + Box-Muller.   */
/* The paper samples Gaussian input perturbations (Sec. III-B, MPPI          */
/* sampling); READING: a counter-based generator keyed by (seed) with the    */
/* counter (sample, step, block, instance).                                   */
/* ------------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    /* S-box: two 32x32->64 multiplications, hi/lo halves mixed with the key */
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k1;
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    /* Weyl key schedule */
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* top 23 bits, centred: (r>>9 + 1/2) / 2^23, never 0 or 1.  23 bits keep the
 * value exactly representable in single precision, so an FP32 implementation
 * draws bit-identical uniforms. */
double orc_uniform23(uint32_t r) { return ((double)(r >> 9) + 0.5) / 8388608.0; }

/* Normals eps[0..K) of sample s at step tau: normal k comes from Philox block
 * k/4 with counter (s, tau, k/4, instance), key (seed lo, seed hi); within a
 * block, Box-Muller maps (u0, u1) -> (n0, n1) and (u2, u3) -> (n2, n3). */
void orc_normals(uint64_t seed, uint32_t instance, uint32_t s, uint32_t tau, int K, double* eps) {
  const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  for (int b = 0; 4 * b < K; ++b) {
    const uint32_t ctr[4] = {s, tau, (uint32_t)b, instance};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    double u[4];
    for (int i = 0; i < 4; ++i) u[i] = orc_uniform23(r[i]);
    double n[4];
    double rad0 = sqrt(-2.0 * log(u[0]));
    double rad1 = sqrt(-2.0 * log(u[2]));
    n[0] = rad0 * cos(2.0 * ORC_PI * u[1]);
    n[1] = rad0 * sin(2.0 * ORC_PI * u[1]);
    n[2] = rad1 * cos(2.0 * ORC_PI * u[3]);
    n[3] = rad1 * sin(2.0 * ORC_PI * u[3]);
    for (int i = 0; i < 4 && 4 * b + i < K; ++i) eps[4 * b + i] = n[i];
  }
}

/* ------------------------------------------------------------------------ */
/* Tractor-trailer kinematics, eq. (6), plus the contour progress psi with   */
/* psi_dot = nu (Sec. IV-B).  State x = [px, py, v, a, th1, th2, delta, psi], */
/* input u = [j, omega, nu].                                                   */
/* ------------------------------------------------------------------------ */

/* continuous drift f_c (input-free part of the vector field); g_c has unit
 * columns on a (jerk), delta (steer rate) and psi (progress rate) */
void orc_drift(const double x[8], const orc_params* p, double f[8]) {
  const double v = x[2], a = x[3], th1 = x[4], th2 = x[5], dl = x[6];
  f[0] = v * cos(th1);
  f[1] = v * sin(th1);
  f[2] = a;
  f[3] = 0.0;
  f[4] = v / p->l1 * tan(dl);
  f[5] = v / p->l2 * (sin(th1 - th2) - p->lh / p->l1 * cos(th1 - th2) * tan(dl));
  f[6] = 0.0;
  f[7] = 0.0;
}

/* explicit Euler step, eq. (6): every right-hand side uses index k */
void orc_step(const double x[8], const double u[3], const orc_params* p, double xn[8]) {
  const double Ts = p->Ts;
  const double px = x[0], py = x[1], v = x[2], a = x[3], th1 = x[4], th2 = x[5], dl = x[6],
               psi = x[7];
  xn[0] = px + Ts * v * cos(th1);
  xn[1] = py + Ts * v * sin(th1);
  xn[2] = v + Ts * a;
  xn[3] = a + Ts * u[0];
  xn[4] = th1 + Ts * v / p->l1 * tan(dl);
  xn[5] = th2 + Ts * v / p->l2 * (sin(th1 - th2) - p->lh / p->l1 * cos(th1 - th2) * tan(dl));
  xn[6] = dl + Ts * u[1];
  xn[7] = psi + Ts * u[2];
}

/* ------------------------------------------------------------------------ */
/* Obstacle barrier, eqs. (16) and (17), exponent e in {2, 4}.                */
/* h = sum_i (d'_i / (m_i + r))^e - 1 with d' = R d the obstacle-frame       */
/* offsets (eq. (16) primes), d = p - p_o(t).  READING: the obstacle moves   */
/* with constant velocity (Assumption 2), p_o(t) = c + v_o t.  hd and hdd    */
/* are the first and second time derivatives of h along the drift (relative  */
/* degree 3: neither depends on the input), and                              */
/* hhat = h + Ts hd + Ts^2/2 hdd (eq. (17)).  Written in the world frame with */
/* the gradient G = R' phi1, Hessian H = R' diag(phi2) R and third           */
/* derivative T3[u, w] = R' (phi3 (R u)(R w)) of h in the position, where    */
/* phi_k is the k-th derivative of y -> (y / (m_i + r))^e per axis; for e = 2 */
/* H = 2Q and T3 = 0.                                                         */
/* ------------------------------------------------------------------------ */

static void mat2_vec(const double Q[2][2], const double v[2], double out[2]) {
  out[0] = Q[0][0] * v[0] + Q[0][1] * v[1];
  out[1] = Q[1][0] * v[0] + Q[1][1] * v[1];
}
static double dot2(const double a[2], const double b[2]) { return a[0] * b[0] + a[1] * b[1]; }
static double ipow(double y, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= y;
  return r;
}

/* Footprint disc (Sec. IV-C: the vehicle body covered by discs of radius r).
 * READING: a disc centre is c = p + A e1 - B f2, with p the tractor's rear
 * axle, e1 = (cos th1, sin th1) and f2 = (cos th2, sin th2): a tractor disc a
 * metres ahead of the rear axle has (A, B) = (a, 0); a trailer disc b metres
 * behind the hitch, which sits lh behind the rear axle (the hitch geometry of
 * eq. (6)), has (A, B) = (-lh, b).  (0, 0) is the rear axle itself, the point
 * eq. (16) uses.  Along the drift (inputs zero) the centre moves with
 *   c'   = v e1 + A w1 e2 - B w2 n2,
 *   c''  = a e1 + v w1 e2 + A (w1' e2 - w1^2 e1) - B (w2' n2 - w2^2 f2),
 * e2, n2 the left normals of e1, f2, w1 = th1' = v tan(delta)/l1 and
 * w2 = th2' = v W(phi, delta) from eq. (6), phi = th1 - th2, and along the
 * drift w1' = a tan(delta)/l1, w2' = a W + v W_phi (w1 - w2). */
typedef struct {
  double c[2], cd[2], cdd[2];            /* centre, velocity, drift acceleration */
  double J0[8][2], J1[8][2], J2[8][2];   /* their partials in the 8 states */
} orc_disc_kin;

static void disc_kinematics(const double x[8], double A, double B, const orc_params* p, orc_disc_kin* k) {
  const double v = x[2], a = x[3], th1 = x[4], th2 = x[5], dl = x[6];
  const double e1[2] = {cos(th1), sin(th1)}, e2[2] = {-sin(th1), cos(th1)};
  const double f2[2] = {cos(th2), sin(th2)}, n2[2] = {-sin(th2), cos(th2)};
  const double tn = tan(dl), sec2 = 1.0 + tn * tn, ch = p->lh / p->l1, phi = th1 - th2;
  const double kd = tn / p->l1, dkd = sec2 / p->l1;
  const double W = (sin(phi) - ch * cos(phi) * tn) / p->l2;
  const double Wp = (cos(phi) + ch * sin(phi) * tn) / p->l2;     /* dW/dphi (and d^2W/dphi^2 = -W) */
  const double Wd = -ch * cos(phi) * sec2 / p->l2;              /* dW/d delta */
  const double Wpd = ch * sin(phi) * sec2 / p->l2;              /* d^2W/dphi d delta */
  const double w1 = v * kd, w2 = v * W;
  const double w1d = a * kd;                                    /* w1' along the drift */
  const double w2d = a * W + v * Wp * (w1 - w2);                /* w2' along the drift */
  memset(k, 0, sizeof(*k));
  for (int i = 0; i < 2; ++i) {
    k->c[i] = x[i] + A * e1[i] - B * f2[i];
    k->cd[i] = v * e1[i] + A * w1 * e2[i] - B * w2 * n2[i];
    k->cdd[i] = a * e1[i] + v * w1 * e2[i] + A * (w1d * e2[i] - w1 * w1 * e1[i]) - B * (w2d * n2[i] - w2 * w2 * f2[i]);
  }
  /* partials of w1, w1', w2, w2' in v, th1, th2, delta (a: w1' and w2' only) */
  const double w2d_v = Wp * (w1 - w2) + v * Wp * (kd - W);
  const double w2d_th1 = a * Wp - v * W * (w1 - w2) - v * v * Wp * Wp;
  const double w2d_dl = a * Wd + v * Wpd * (w1 - w2) + v * Wp * (v * dkd - v * Wd);
  for (int i = 0; i < 2; ++i) {
    /* position: p, th1 (e1), th2 (f2) */
    k->J0[0][i] = (i == 0);
    k->J0[1][i] = (i == 1);
    k->J0[4][i] = A * e2[i];
    k->J0[5][i] = -B * n2[i];
    /* velocity */
    k->J1[2][i] = e1[i] + A * kd * e2[i] - B * W * n2[i];
    k->J1[4][i] = v * e2[i] - A * w1 * e1[i] - B * v * Wp * n2[i];
    k->J1[5][i] = B * v * Wp * n2[i] + B * w2 * f2[i];
    k->J1[6][i] = A * v * dkd * e2[i] - B * v * Wd * n2[i];
    /* drift acceleration */
    k->J2[2][i] = 2.0 * w1 * e2[i] - 2.0 * A * w1 * kd * e1[i] - B * (w2d_v * n2[i] - 2.0 * w2 * W * f2[i]);
    k->J2[3][i] = e1[i] + A * kd * e2[i] - B * W * n2[i];
    k->J2[4][i] = a * e2[i] - v * w1 * e1[i] + A * (-w1d * e1[i] - w1 * w1 * e2[i]) -
                  B * (w2d_th1 * n2[i] - 2.0 * w2 * v * Wp * f2[i]);
    k->J2[5][i] = -B * (-w2d_th1 * n2[i] - w2d * f2[i] + 2.0 * w2 * v * Wp * f2[i] - w2 * w2 * n2[i]);
    k->J2[6][i] = v * v * dkd * e2[i] + A * (a * dkd * e2[i] - 2.0 * w1 * v * dkd * e1[i]) -
                  B * (w2d_dl * n2[i] - 2.0 * w2 * v * Wd * f2[i]);
  }
}

/* the barrier of eqs. (16)-(17) for obstacle o around the disc centre (A, B) */
void orc_disc_barrier(const double x[8], double t, const orc_obstacle* o, double A, double B,
                      const orc_params* p, orc_barrier* out) {
  const double Ts = p->Ts;
  const int e = (int)o->e;
  const double co = cos(o->heading), so = sin(o->heading);
  const double R[2][2] = {{co, so}, {-so, co}};          /* world -> obstacle frame */
  const double rho[2] = {1.0 / (o->mx + p->r_disc), 1.0 / (o->my + p->r_disc)};
  orc_disc_kin K;
  disc_kinematics(x, A, B, p, &K);

  const double vo[2] = {o->vx, o->vy};
  const double d[2] = {K.c[0] - (o->cx + o->vx * t), K.c[1] - (o->cy + o->vy * t)};
  /* d_dot and d_ddot along the drift (the obstacle moves at constant velocity) */
  const double dd[2] = {K.cd[0] - vo[0], K.cd[1] - vo[1]};
  const double* ddd = K.cdd;

  /* per-axis derivatives of phi in the obstacle frame */
  double dp[2], f0 = -1.0, f1[2], f2[2], f3[2];
  mat2_vec(R, d, dp);
  for (int i = 0; i < 2; ++i) {
    const double ri = ipow(rho[i], e);
    f0 += ri * ipow(dp[i], e);
    f1[i] = e * ri * ipow(dp[i], e - 1);
    f2[i] = e * (e - 1) * ri * ipow(dp[i], e - 2);
    f3[i] = (e >= 3) ? e * (e - 1) * (e - 2) * ri * ipow(dp[i], e - 3) : 0.0;
  }
  /* world-frame gradient, Hessian and third-derivative contraction T3[dd, dd] */
  double G[2], H[2][2];
  G[0] = R[0][0] * f1[0] + R[1][0] * f1[1];
  G[1] = R[0][1] * f1[0] + R[1][1] * f1[1];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) H[i][j] = R[0][i] * f2[0] * R[0][j] + R[1][i] * f2[1] * R[1][j];
  double Rdd[2], T3dd[2];
  mat2_vec(R, dd, Rdd);
  T3dd[0] = R[0][0] * f3[0] * Rdd[0] * Rdd[0] + R[1][0] * f3[1] * Rdd[1] * Rdd[1];
  T3dd[1] = R[0][1] * f3[0] * Rdd[0] * Rdd[0] + R[1][1] * f3[1] * Rdd[1] * Rdd[1];
  double Hdd[2], Hddd[2];
  mat2_vec(H, dd, Hdd);
  mat2_vec(H, ddd, Hddd);

  const double h = f0;
  const double hd = dot2(G, dd);
  const double hdd = dot2(dd, Hdd) + dot2(G, ddd);
  out->h = h;
  out->hd = hd;
  out->hdd = hdd;
  out->hhat = h + Ts * hd + 0.5 * Ts * Ts * hdd;

  /* partial derivatives of h, hd, hdd (chain rule through c, c', c'') */
  for (int i = 0; i < 8; ++i) {
    const double* j0 = K.J0[i];
    const double* j1 = K.J1[i];
    const double* j2 = K.J2[i];
    double Hj0[2];
    mat2_vec(H, j0, Hj0);
    const double gh = dot2(G, j0);
    const double ghd = dot2(dd, Hj0) + dot2(G, j1);
    const double ghdd = dot2(T3dd, j0) + 2.0 * dot2(Hdd, j1) + dot2(ddd, Hj0) + dot2(G, j2);
    out->grad[i] = gh + Ts * ghd + 0.5 * Ts * Ts * ghdd;
  }
  /* time partials: d depends on t through -v_o t */
  const double th = -dot2(vo, G);
  const double thd = -dot2(vo, Hdd);
  const double thdd = -(T3dd[0] * vo[0] + T3dd[1] * vo[1]) - dot2(vo, Hddd);
  out->dt = th + Ts * thd + 0.5 * Ts * Ts * thdd;
}

/* eq. (16) as printed: the rear axle's point */
void orc_obstacle_barrier(const double x[8], double t, const orc_obstacle* o, const orc_params* p,
                          orc_barrier* out) {
  orc_disc_barrier(x, t, o, 0.0, 0.0, p, out);
}

/* disc k of the footprint in row order: the tractor's, then the trailer's */
int orc_num_discs(const orc_params* p) { return p->n_disc_tractor + p->n_disc_trailer; }
void orc_disc(const orc_params* p, int k, double* A, double* B) {
  if (k < p->n_disc_tractor) {
    *A = p->disc_tractor[k];
    *B = 0.0;
  } else {
    *A = -p->lh;
    *B = p->disc_trailer[k - p->n_disc_tractor];
  }
}

/* ------------------------------------------------------------------------ */
/* Hitch-angle barrier, eq. (18): h = dth_max - kappa v - |th2 - th1|.        */
/* READING: the kink of |.| is split into two smooth rows                     */
/*   h_s = dth_max - kappa v - s (th2 - th1),  s = +1, -1,                    */
/* whose intersection is the same safe set.  The hitch barrier has relative   */
/* degree 2, so (by the same rule eq. (17) applies to the degree-3 obstacle   */
/* barrier) it is expanded to first order: hhat = h + Ts hd.                  */
/* ------------------------------------------------------------------------ */
void orc_hitch_barrier(const double x[8], int sign, const orc_params* p, orc_barrier* out) {
  const double v = x[2], a = x[3], th1 = x[4], th2 = x[5], dl = x[6];
  const double s = (double)sign;
  const double Ts = p->Ts;
  const double phi = th1 - th2;
  const double tn = tan(dl), sec2 = 1.0 + tn * tn;
  const double c = p->lh / p->l1;
  /* heading rates along the drift, eq. (6) */
  const double w1 = v / p->l1 * tn;
  const double w2 = v / p->l2 * (sin(phi) - c * cos(phi) * tn);
  /* partials of w1, w2 with respect to v, th1, th2, delta */
  const double w1_v = tn / p->l1, w1_dl = v / p->l1 * sec2;
  const double w2_v = (sin(phi) - c * cos(phi) * tn) / p->l2;
  const double w2_th1 = v / p->l2 * (cos(phi) + c * sin(phi) * tn);
  const double w2_th2 = -w2_th1;
  const double w2_dl = v / p->l2 * (-c * cos(phi) * sec2);

  const double h = p->dtheta_max - p->kappa * v - s * (th2 - th1);
  const double hd = -p->kappa * a - s * (w2 - w1);
  out->h = h;
  out->hd = hd;
  out->hdd = 0.0;
  out->hhat = h + Ts * hd;

  double g[8] = {0};
  /* dh */
  g[2] += -p->kappa;
  g[4] += s;
  g[5] += -s;
  /* Ts * dhd */
  g[2] += Ts * (-s * (w2_v - w1_v));
  g[3] += Ts * (-p->kappa);
  g[4] += Ts * (-s * w2_th1);
  g[5] += Ts * (-s * w2_th2);
  g[6] += Ts * (-s * (w2_dl - w1_dl));
  memcpy(out->grad, g, sizeof(g));
  out->dt = 0.0;
}

/* ------------------------------------------------------------------------ */
/* Constraint rows of eq. (9) at state x, time t.                             */
/* Row i:  Lf_i + g_i u = -(alpha_i + u^alpha_i) hhat_i, with                 */
/*   Lf_i = Ts (grad hhat . f_c + d hhat/dt)   (f = Ts f_c, Sec. III-A)      */
/*   g_i  = Ts (d hhat/da, d hhat/d delta)     (jerk, steer-rate columns;     */
/*          the progress-rate column is zero because hhat does not involve psi)*/
/* Order: hitch (+), hitch (-) (absent with ORC_HITCH_OFF), then one row per */
/* (footprint disc, obstacle), disc by disc (orc_disc), obstacles as given.  */
/* READING (guard against a singular A M^-1 A'): hhat is replaced by           */
/* copysign(max(|hhat|, h_eps), hhat), with 0 mapped to +h_eps.                */
/* ------------------------------------------------------------------------ */
int orc_num_rows(const orc_problem* pr, const orc_params* p) {
  return pr->n_obs * orc_num_discs(p) + ((pr->flags & ORC_HITCH_OFF) ? 0 : 2);
}

/* Normals drawn per (sample, step): 0..2 perturb (j, omega, nu); 3 and 4 are
 * the auxiliary inputs of the hitch rows (+, -); 5 + k n_obs + o that of the
 * row of disc k and obstacle o.  The numbering does not depend on
 * ORC_HITCH_OFF (3 and 4 are then unused). */
int orc_num_normals(const orc_problem* pr, const orc_params* p) { return 5 + pr->n_obs * orc_num_discs(p); }

/* normal index of row i in the order produced by orc_rows */
static int row_normal(const orc_problem* pr, int i) {
  if (pr->flags & ORC_HITCH_OFF) return 5 + i;
  return 3 + i;
}

static void row_from_barrier(const orc_barrier* B, const double f[8], const orc_params* p,
                             double* hraw, double* hh, double* G2, double* Lf) {
  double lf = B->dt;
  for (int k = 0; k < 8; ++k) lf += B->grad[k] * f[k];
  *Lf = p->Ts * lf;
  G2[0] = p->Ts * B->grad[3];
  G2[1] = p->Ts * B->grad[6];
  *hraw = B->hhat;
  double m = fabs(B->hhat);
  if (m < p->h_eps) m = p->h_eps;
  *hh = (B->hhat < 0.0) ? -m : m;
}

void orc_rows(const orc_problem* pr, const orc_params* p, const double x[8], double t,
              double* hraw, double* hh, double* G, double* Lf) {
  double f[8];
  orc_drift(x, p, f);
  int i = 0;
  if (!(pr->flags & ORC_HITCH_OFF)) {
    for (int sgn = 1; sgn >= -1; sgn -= 2, ++i) {
      orc_barrier B;
      orc_hitch_barrier(x, sgn, p, &B);
      row_from_barrier(&B, f, p, &hraw[i], &hh[i], &G[2 * i], &Lf[i]);
    }
  }
  for (int k = 0; k < orc_num_discs(p); ++k) {
    double A, Bd;
    orc_disc(p, k, &A, &Bd);
    for (int o = 0; o < pr->n_obs; ++o, ++i) {
      orc_barrier B;
      orc_disc_barrier(x, t, &pr->obs[o], A, Bd, p, &B);
      row_from_barrier(&B, f, p, &hraw[i], &hh[i], &G[2 * i], &Lf[i]);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Soft-bound projection, eqs. (11) and (12), solved densely.                 */
/* z = [j, omega, u^alpha_1..nc]; W = Diag(W_j, W_w, W_a I); M = W + rho I;   */
/* p = W z_des + rho/2 (z_lo + z_hi); A = [G | diag(hhat)]; b_i = -Lf_i -      */
/* alpha_i hhat_i (eq. (9) moved to A z = b form).                             */
/* READING: the alpha bounds act on the next barrier rate, so for u^alpha_i  */
/* z_lo = alpha_lo - alpha_i and z_hi = alpha_hi - alpha_i.                    */
/* z* = M^-1 [p - A' (A M^-1 A')^-1 (A M^-1 p - b)]; the nc x nc system is     */
/* solved by Gaussian elimination with partial pivoting.                      */
/* ------------------------------------------------------------------------ */
static int lu_solve(int n, double* K, double* rhs) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(K[r * n + c]) > fabs(K[piv * n + c])) piv = r;
    if (K[piv * n + c] == 0.0) return -1;
    if (piv != c) {
      for (int k = 0; k < n; ++k) {
        double tmp = K[c * n + k];
        K[c * n + k] = K[piv * n + k];
        K[piv * n + k] = tmp;
      }
      double tmp = rhs[c];
      rhs[c] = rhs[piv];
      rhs[piv] = tmp;
    }
    for (int r = c + 1; r < n; ++r) {
      double f = K[r * n + c] / K[c * n + c];
      for (int k = c; k < n; ++k) K[r * n + k] -= f * K[c * n + k];
      rhs[r] -= f * rhs[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double s = rhs[r];
    for (int k = r + 1; k < n; ++k) s -= K[r * n + k] * rhs[k];
    rhs[r] = s / K[r * n + r];
  }
  return 0;
}

int orc_project(int nc, const double* zdes, const double* alpha, const double* hh, const double* G,
                const double* b, const orc_params* p, double* zstar) {
  const int nz = 2 + nc;
  double* Wd = (double*)malloc(sizeof(double) * nz);
  double* Md = (double*)malloc(sizeof(double) * nz);
  double* pv = (double*)malloc(sizeof(double) * nz);
  double* A = (double*)calloc((size_t)nc * nz + 1, sizeof(double));
  double* K = (double*)malloc(sizeof(double) * (nc * nc + 1));
  double* lam = (double*)malloc(sizeof(double) * (nc + 1));
  int rc = 0;
  Wd[0] = p->W_j;
  Wd[1] = p->W_w;
  for (int i = 0; i < nc; ++i) Wd[2 + i] = p->W_a;
  for (int k = 0; k < nz; ++k) Md[k] = Wd[k] + p->rho;
  /* bounds */
  for (int k = 0; k < nz; ++k) {
    double lo, hi;
    if (k == 0) { lo = p->j_lo; hi = p->j_hi; }
    else if (k == 1) { lo = p->w_lo; hi = p->w_hi; }
    else { lo = p->alpha_lo - alpha[k - 2]; hi = p->alpha_hi - alpha[k - 2]; }
    pv[k] = Wd[k] * zdes[k] + 0.5 * p->rho * (lo + hi);
  }
  for (int i = 0; i < nc; ++i) {
    A[i * nz + 0] = G[2 * i + 0];
    A[i * nz + 1] = G[2 * i + 1];
    A[i * nz + 2 + i] = hh[i];
  }
  /* K = A M^-1 A',  lam = A M^-1 p - b */
  for (int i = 0; i < nc; ++i) {
    for (int j = 0; j < nc; ++j) {
      double s = 0.0;
      for (int k = 0; k < nz; ++k) s += A[i * nz + k] * A[j * nz + k] / Md[k];
      K[i * nc + j] = s;
    }
    double s = 0.0;
    for (int k = 0; k < nz; ++k) s += A[i * nz + k] * pv[k] / Md[k];
    lam[i] = s - b[i];
  }
  if (nc > 0 && lu_solve(nc, K, lam) != 0) rc = -1;
  for (int k = 0; k < nz; ++k) {
    double s = pv[k];
    for (int i = 0; i < nc; ++i) s -= A[i * nz + k] * lam[i];
    zstar[k] = s / Md[k];
  }
  free(Wd); free(Md); free(pv); free(A); free(K); free(lam);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Contouring cost, eqs. (13)-(15).                                           */
/* READING: the reference zeta(psi) is the table of waypoints every ds metres */
/* (the spline fit happens when the path is built); between waypoints x, y    */
/* are interpolated linearly and headings by the wrapped difference; psi      */
/* outside [0, (n-1) ds] uses the end waypoint.                               */
/* ------------------------------------------------------------------------ */
double orc_wrap(double a) { return a - 2.0 * ORC_PI * nearbyint(a / (2.0 * ORC_PI)); }

void orc_reference(const double* path, int n, double ds, double psi, double ref[4]) {
  const double f = psi / ds;
  double fi = floor(f);
  if (fi < 0.0) fi = 0.0;
  if (fi > (double)(n - 2)) fi = (double)(n - 2);
  const int i = (int)fi;
  double t = f - fi;
  if (t < 0.0) t = 0.0;
  if (t > 1.0) t = 1.0;
  const double* A = path + 4 * i;
  const double* B = path + 4 * (i + 1);
  ref[0] = A[0] + t * (B[0] - A[0]);
  ref[1] = A[1] + t * (B[1] - A[1]);
  ref[2] = A[2] + t * orc_wrap(B[2] - A[2]);
  ref[3] = A[3] + t * orc_wrap(B[3] - A[3]);
}

static double tracking_terms(const double x[8], const double* path, int n, double ds,
                             const orc_params* p) {
  double ref[4];
  orc_reference(path, n, ds, x[7], ref);
  const double ex = x[0] - ref[0], ey = x[1] - ref[1];
  const double ec = sin(ref[2]) * ex - cos(ref[2]) * ey;    /* eq. (14) */
  const double el = -cos(ref[2]) * ex - sin(ref[2]) * ey;   /* eq. (15) */
  const double eth1 = orc_wrap(x[4] - ref[2]);
  const double eth2 = orc_wrap(x[5] - ref[3]);
  return p->Qc * ec * ec + p->Ql * el * el + p->Qth1 * eth1 * eth1 + p->Qth2 * eth2 * eth2;
}

/* r(x, u, psi), eq. (13); READING: the effort term covers jerk and steer rate */
double orc_stage_cost(const double x[8], const double u[3], const double* path, int n, double ds,
                      const orc_params* p) {
  const double prog = p->nu_bar - u[2];
  return tracking_terms(x, path, n, ds, p) + p->R_j * u[0] * u[0] + p->R_w * u[1] * u[1] +
         p->mu * prog * prog;
}

/* Collision-penalty baseline (Sec. V, the second MPPI baseline; the paper   */
/* gives no formula).  READING: w_col * sum_o max(0, -h_o(x, t))^2 with h_o   */
/* the obstacle function of eq. (16) (exponent e = 2 or 4, as the obstacle   */
/* has it) at the current state and time, added to the stage cost of every   */
/* step and to the terminal cost.                                            */
/* With several footprint discs every (disc, obstacle) pair is penalised.     */
double orc_collision_penalty(const double x[8], double t, const orc_obstacle* obs, int n_obs, const orc_params* p) {
  double pen = 0.0;
  for (int k = 0; k < orc_num_discs(p); ++k) {
    double A, Bd;
    orc_disc(p, k, &A, &Bd);
    for (int o = 0; o < n_obs; ++o) {
      orc_barrier B;
      orc_disc_barrier(x, t, &obs[o], A, Bd, p, &B);
      if (B.h < 0.0) pen += B.h * B.h;
    }
  }
  return p->w_col * pen;
}

/* READING: r_N (eq. (7)) is the tracking part of eq. (13) at the final state */
double orc_terminal_cost(const double x[8], const double* path, int n, double ds, const orc_params* p) {
  return tracking_terms(x, path, n, ds, p);
}

/* ------------------------------------------------------------------------ */
/* One rollout (Sec. IV-A, with the MPPI sampling of Sec. III-B).             */
/* For tau = 0..T-1: draw eps (or take it from `eps`), form                   */
/*   u_des = u_nom[tau] + sigma * eps[0:3],  u~alpha_i = sigma_a eps[n(i)]    */
/*   (n(i) the normal of row i, see orc_num_normals),                          */
/* project z_des = [j, omega, u~alpha] with eq. (12), apply u* = (j*, w*, nu)  */
/* (READING: the progress rate is not projected), add r(x_tau, u*_tau),       */
/* step eq. (6), update alpha_{tau+1} = alpha_tau + u*alpha.                  */
/* J = sum_tau r + r_N(x_T).  alpha starts at alpha0 for every row.           */
/* eps, when given, is T*(5+n_obs) for this sample.                            */
/* ------------------------------------------------------------------------ */
double orc_rollout(const orc_problem* pr, const orc_params* p, uint32_t s, const double* eps,
                   double* useq, double* traj, double* alphas) {
  const int nc = orc_num_rows(pr, p);
  const int K = orc_num_normals(pr, p);
  const int guided = !(pr->flags & ORC_GUIDANCE_OFF);
  double x[8];
  memcpy(x, pr->x0, sizeof(x));
  double* alpha = (double*)malloc(sizeof(double) * (nc + 1));
  double* e = (double*)malloc(sizeof(double) * K);
  double* hraw = (double*)malloc(sizeof(double) * (nc + 1));
  double* hh = (double*)malloc(sizeof(double) * (nc + 1));
  double* G = (double*)malloc(sizeof(double) * (2 * nc + 1));
  double* Lf = (double*)malloc(sizeof(double) * (nc + 1));
  double* b = (double*)malloc(sizeof(double) * (nc + 1));
  double* zd = (double*)malloc(sizeof(double) * (2 + nc));
  double* zs = (double*)malloc(sizeof(double) * (2 + nc));
  for (int i = 0; i < nc; ++i) alpha[i] = p->alpha0;
  if (traj) memcpy(traj, x, sizeof(x));
  double J = 0.0;
  for (int tau = 0; tau < pr->T; ++tau) {
    const double t = pr->t0 + tau * p->Ts;
    if (eps) memcpy(e, eps + (size_t)tau * K, sizeof(double) * K);
    else orc_normals(pr->seed, pr->instance, s, (uint32_t)tau, K, e);
    double u[3];
    u[0] = pr->u_nom[3 * tau + 0] + p->sigma_j * e[0];
    u[1] = pr->u_nom[3 * tau + 1] + p->sigma_w * e[1];
    u[2] = pr->u_nom[3 * tau + 2] + p->sigma_nu * e[2];
    if (guided) {
      orc_rows(pr, p, x, t, hraw, hh, G, Lf);
      for (int i = 0; i < nc; ++i) b[i] = -Lf[i] - alpha[i] * hh[i];
      zd[0] = u[0];
      zd[1] = u[1];
      for (int i = 0; i < nc; ++i) zd[2 + i] = p->sigma_a * e[row_normal(pr, i)];
      orc_project(nc, zd, alpha, hh, G, b, p, zs);
      u[0] = zs[0];
      u[1] = zs[1];
    }
    J += orc_stage_cost(x, u, pr->path, pr->n_path, pr->ds, p);
    if (pr->flags & ORC_COLLISION_PENALTY) J += orc_collision_penalty(x, t, pr->obs, pr->n_obs, p);
    if (useq) memcpy(useq + 3 * tau, u, sizeof(u));
    double xn[8];
    orc_step(x, u, p, xn);
    memcpy(x, xn, sizeof(x));
    if (guided)
      for (int i = 0; i < nc; ++i) alpha[i] += zs[2 + i];
    if (traj) memcpy(traj + 8 * (tau + 1), x, sizeof(x));
    if (alphas) memcpy(alphas + (size_t)nc * tau, alpha, sizeof(double) * nc);
  }
  J += orc_terminal_cost(x, pr->path, pr->n_path, pr->ds, p);
  if (pr->flags & ORC_COLLISION_PENALTY)
    J += orc_collision_penalty(x, pr->t0 + pr->T * p->Ts, pr->obs, pr->n_obs, p);
  free(alpha); free(e); free(hraw); free(hh); free(G); free(Lf); free(b); free(zd); free(zs);
  if (!isfinite(J)) J = INFINITY;
  return J;
}

void orc_rollout_samples(const orc_problem* pr, const orc_params* p, const uint32_t* ids, int n,
                         int nthreads, double* J, double* useq) {
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 4)
  for (int i = 0; i < n; ++i)
    J[i] = orc_rollout(pr, p, ids[i], NULL, useq ? useq + (size_t)i * 3 * pr->T : NULL, NULL, NULL);
}

/* ------------------------------------------------------------------------ */
/* Importance weights (Sec. III-B): gamma_s = exp(-(J_s - min J)/lambda),     */
/* normalised.  READING: lambda divides (a temperature); a non-finite cost    */
/* gets weight 0; if no cost is finite, return -1.                            */
/* ------------------------------------------------------------------------ */
int orc_weights(const double* J, int S, double lambda, double* wbar, double* m_out, double* Z_out) {
  double m = INFINITY;
  for (int s = 0; s < S; ++s)
    if (isfinite(J[s]) && J[s] < m) m = J[s];
  if (!isfinite(m)) {
    for (int s = 0; s < S; ++s) wbar[s] = 0.0;
    if (m_out) *m_out = m;
    if (Z_out) *Z_out = 0.0;
    return -1;
  }
  double Z = 0.0;
  for (int s = 0; s < S; ++s) {
    wbar[s] = isfinite(J[s]) ? exp(-(J[s] - m) / lambda) : 0.0;
    Z += wbar[s];
  }
  for (int s = 0; s < S; ++s) wbar[s] /= Z;
  if (m_out) *m_out = m;
  if (Z_out) *Z_out = Z;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* One control update: S rollouts, weights, eq. (5) on the applied inputs.    */
/* READING: the average is taken over the projected (applied) sequences.      */
/* Returns 0, or -1 when every cost is non-finite (then U_new = u_nom).       */
/* stats[0..2] = (min J, sum gamma, effective sample size 1/sum wbar^2).       */
/* ------------------------------------------------------------------------ */
int orc_solve(const orc_problem* pr, const orc_params* p, int nthreads, const double* eps,
              double* U_new, double* J, double* wbar, double* useq_all, double* stats) {
  const int S = pr->S, T = pr->T;
  const int K = orc_num_normals(pr, p);
  int own = 0;
  if (!useq_all) {
    useq_all = (double*)malloc(sizeof(double) * (size_t)S * T * 3);
    own = 1;
  }
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 4)
  for (int s = 0; s < S; ++s)
    J[s] = orc_rollout(pr, p, (uint32_t)s, eps ? eps + (size_t)s * T * K : NULL,
                       useq_all + (size_t)s * T * 3, NULL, NULL);
  double m = 0, Z = 0;
  int rc = orc_weights(J, S, pr->lambda, wbar, &m, &Z);
  if (rc != 0) {
    memcpy(U_new, pr->u_nom, sizeof(double) * 3 * T);
  } else {
    for (int k = 0; k < 3 * T; ++k) U_new[k] = 0.0;
    for (int s = 0; s < S; ++s)
      for (int k = 0; k < 3 * T; ++k) U_new[k] += wbar[s] * useq_all[(size_t)s * T * 3 + k];
  }
  if (stats) {
    double w2 = 0.0;
    for (int s = 0; s < S; ++s) w2 += wbar[s] * wbar[s];
    stats[0] = m;
    stats[1] = Z;
    stats[2] = (w2 > 0.0) ? 1.0 / w2 : 0.0;
  }
  if (own) free(useq_all);
  return rc;
}

/* Closed-loop plant for the reverse-parking workload: the first averaged input,
 * jerk and steer rate clamped to the actuator bounds of Sec. V, applied with
 * eq. (6); the virtual progress state advances by Ts nu. */
/* ------------------------------------------------------------------------ */
/* Hitch-angle stabiliser (Sec. IV-D, eq. (19)): u* = argmin over the input  */
/* box of ||u - u_ref||^2_{Q_h} subject to the discrete CBF condition of the */
/* hitch barrier, on (j, omega).  READINGS: the barrier has relative degree  */
/* 2 in (j, omega), so the condition uses the same first-order expansion as  */
/* the rollout rows, hhat = h + Ts hdot, one row per sign of the hitch angle;*/
/* the class-K term carries the standard sign, Lf + g u >= -alpha_h hhat;    */
/* U is the hard input box [j_lo, j_hi] x [w_lo, w_hi].  Solved exactly by    */
/* enumerating the active sets of at most two of the six constraints and     */
/* keeping the KKT point (primal and dual feasible).  If no input satisfies   */
/* the constraints, the reference clipped to the box is returned (status 1). */
/* ------------------------------------------------------------------------ */
int orc_hitch_qp(const double x[8], const double uref[2], const orc_params* p, double u_out[2]) {
  double A[6][2], c[6];
  double f[8];
  orc_drift(x, p, f);
  int n = 0;
  for (int sgn = 1; sgn >= -1; sgn -= 2, ++n) {
    orc_barrier B;
    orc_hitch_barrier(x, sgn, p, &B);
    double hraw, hh, G2[2], Lf;
    row_from_barrier(&B, f, p, &hraw, &hh, G2, &Lf);
    A[n][0] = G2[0];
    A[n][1] = G2[1];
    c[n] = -p->alpha_h * hraw - Lf;
  }
  const double box[4][3] = {{1, 0, p->j_lo}, {-1, 0, -p->j_hi}, {0, 1, p->w_lo}, {0, -1, -p->w_hi}};
  for (int k = 0; k < 4; ++k, ++n) {
    A[n][0] = box[k][0];
    A[n][1] = box[k][1];
    c[n] = box[k][2];
  }
  const double q[2] = {p->qh_j, p->qh_w};
  double best = INFINITY, bu[2] = {0, 0};
  /* active set of size 0 */
  int cand = 0;
  double U[1 + 6 + 15][2], L[1 + 6 + 15][2];
  int act[1 + 6 + 15][2], nact[1 + 6 + 15];
  U[cand][0] = uref[0];
  U[cand][1] = uref[1];
  nact[cand++] = 0;
  /* size 1: u = uref + Q^-1 a lam, a'u = c */
  for (int i = 0; i < n; ++i) {
    const double aQa = A[i][0] * A[i][0] / q[0] + A[i][1] * A[i][1] / q[1];
    if (!(aQa > 0.0)) continue;
    const double lam = (c[i] - (A[i][0] * uref[0] + A[i][1] * uref[1])) / aQa;
    U[cand][0] = uref[0] + A[i][0] / q[0] * lam;
    U[cand][1] = uref[1] + A[i][1] / q[1] * lam;
    L[cand][0] = lam;
    act[cand][0] = i;
    nact[cand++] = 1;
  }
  /* size 2: M lam = c_S - A_S uref, M_ik = a_i' Q^-1 a_k */
  for (int i = 0; i < n; ++i) {
    for (int k = i + 1; k < n; ++k) {
      const double m00 = A[i][0] * A[i][0] / q[0] + A[i][1] * A[i][1] / q[1];
      const double m01 = A[i][0] * A[k][0] / q[0] + A[i][1] * A[k][1] / q[1];
      const double m11 = A[k][0] * A[k][0] / q[0] + A[k][1] * A[k][1] / q[1];
      const double det = m00 * m11 - m01 * m01;
      if (!(fabs(det) > 1e-14 * (m00 * m11 + 1e-300))) continue;
      const double r0 = c[i] - (A[i][0] * uref[0] + A[i][1] * uref[1]);
      const double r1 = c[k] - (A[k][0] * uref[0] + A[k][1] * uref[1]);
      const double l0 = (m11 * r0 - m01 * r1) / det, l1 = (m00 * r1 - m01 * r0) / det;
      U[cand][0] = uref[0] + (A[i][0] * l0 + A[k][0] * l1) / q[0];
      U[cand][1] = uref[1] + (A[i][1] * l0 + A[k][1] * l1) / q[1];
      L[cand][0] = l0;
      L[cand][1] = l1;
      act[cand][0] = i;
      act[cand][1] = k;
      nact[cand++] = 2;
    }
  }
  for (int z = 0; z < cand; ++z) {
    int ok = 1;
    for (int j = 0; j < nact[z]; ++j)
      if (L[z][j] < -1e-12) ok = 0;                      /* dual feasibility */
    for (int i = 0; i < n && ok; ++i) {
      const double r = A[i][0] * U[z][0] + A[i][1] * U[z][1] - c[i];
      const double scale = fabs(c[i]) + fabs(A[i][0] * U[z][0]) + fabs(A[i][1] * U[z][1]) + 1e-300;
      if (r < -1e-10 * scale) ok = 0;                    /* primal feasibility */
    }
    if (!ok) continue;
    const double obj = q[0] * (U[z][0] - uref[0]) * (U[z][0] - uref[0]) + q[1] * (U[z][1] - uref[1]) * (U[z][1] - uref[1]);
    if (obj < best) {
      best = obj;
      bu[0] = U[z][0];
      bu[1] = U[z][1];
    }
  }
  if (best < INFINITY) {
    u_out[0] = bu[0];
    u_out[1] = bu[1];
    return 0;
  }
  u_out[0] = fmin(fmax(uref[0], p->j_lo), p->j_hi);
  u_out[1] = fmin(fmax(uref[1], p->w_lo), p->w_hi);
  return 1;
}

/* closed-loop plant step with the stabiliser applied to the averaged input */
void orc_plant_step_qp(const double x[8], const double U0[3], const orc_params* p, double xn[8]) {
  double u[3];
  orc_hitch_qp(x, U0, p, u);
  u[2] = U0[2];
  orc_step(x, u, p, xn);
}

void orc_plant_step(const double x[8], const double U0[3], const orc_params* p, double xn[8]) {
  double u[3] = {U0[0], U0[1], U0[2]};
  if (u[0] < p->j_lo) u[0] = p->j_lo;
  if (u[0] > p->j_hi) u[0] = p->j_hi;
  if (u[1] < p->w_lo) u[1] = p->w_lo;
  if (u[1] > p->w_hi) u[1] = p->w_hi;
  orc_step(x, u, p, xn);
}
