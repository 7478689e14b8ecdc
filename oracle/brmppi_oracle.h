/*
 * FP64 CPU oracle for one BR-MPPI control update -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may load
 * or call this code.  It shares nothing with the HIP path (no headers, helpers
 * or constants); its own structs are declared here.
 *
 * Paper: "GPU-Accelerated Barrier-Rate Guided MPPI Control for Tractor-Trailer
 * Systems" (arXiv 2508.05773).  Every function cites the passage it follows.
 */
#ifndef BRMPPI_ORACLE_H
#define BRMPPI_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double Ts, l1, lh, l2, dtheta_max, kappa, r_disc;
  double Qc, Ql, Qth1, Qth2, R_j, R_w, mu, nu_bar;
  double W_j, W_w, W_a, rho, j_lo, j_hi, w_lo, w_hi;
  double alpha0, alpha_lo, alpha_hi, sigma_j, sigma_w, sigma_nu, sigma_a;
  double h_eps;
  double w_col;                /* collision-penalty weight (baseline flag only) */
  double qh_j, qh_w, alpha_h;  /* hitch-angle stabiliser QP, eq. (19): Q_h, class-K rate */
  /* footprint discs (Sec. IV-C): tractor discs a metres ahead of the rear axle,
   * trailer discs b metres behind the hitch; one barrier row per (disc, obstacle) */
  double disc_tractor[4], disc_trailer[4];
  int n_disc_tractor, n_disc_trailer;
} orc_params;

/* obstacle: centre, semi-axes, orientation, exponent, constant velocity */
typedef struct { double cx, cy, mx, my, heading, e, vx, vy; } orc_obstacle;

enum { ORC_GUIDANCE_OFF = 1, ORC_HITCH_OFF = 2, ORC_COLLISION_PENALTY = 16 };

typedef struct {
  int S, T;
  double x0[8];                /* px, py, v, a, theta1, theta2, delta, psi */
  const double* u_nom;         /* T*3 */
  const orc_obstacle* obs;
  int n_obs;
  const double* path;          /* n_path*4: x, y, theta1_ref, theta2_ref */
  int n_path;
  double ds, t0, lambda;
  uint64_t seed;
  uint32_t instance;
  int flags;
} orc_problem;

/* one barrier evaluated at a state: the Taylor barrier hhat, its parts, and
 * its gradient with respect to the 8 states and to time */
typedef struct {
  double h, hd, hdd, hhat;
  double grad[8];
  double dt;
} orc_barrier;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_uniform23(uint32_t r);
void orc_normals(uint64_t seed, uint32_t instance, uint32_t s, uint32_t tau, int K, double* eps);

void orc_drift(const double x[8], const orc_params* p, double f[8]);
void orc_step(const double x[8], const double u[3], const orc_params* p, double xn[8]);

void orc_obstacle_barrier(const double x[8], double t, const orc_obstacle* o, const orc_params* p,
                          orc_barrier* out);
void orc_hitch_barrier(const double x[8], int sign, const orc_params* p, orc_barrier* out);
void orc_disc_barrier(const double x[8], double t, const orc_obstacle* o, double A, double B,
                      const orc_params* p, orc_barrier* out);
int orc_num_discs(const orc_params* p);
void orc_disc(const orc_params* p, int k, double* A, double* B);

int orc_num_rows(const orc_problem* pr, const orc_params* p);
int orc_num_normals(const orc_problem* pr, const orc_params* p);
void orc_rows(const orc_problem* pr, const orc_params* p, const double x[8], double t,
              double* hraw, double* hh, double* G, double* Lf);

int orc_project(int nc, const double* zdes, const double* alpha, const double* hh, const double* G,
                const double* b, const orc_params* p, double* zstar);

void orc_reference(const double* path, int n, double ds, double psi, double ref[4]);
double orc_wrap(double a);
double orc_stage_cost(const double x[8], const double u[3], const double* path, int n, double ds,
                      const orc_params* p);
double orc_terminal_cost(const double x[8], const double* path, int n, double ds, const orc_params* p);
int orc_hitch_qp(const double x[8], const double uref[2], const orc_params* p, double u_out[2]);
void orc_plant_step_qp(const double x[8], const double U0[3], const orc_params* p, double xn[8]);
double orc_collision_penalty(const double x[8], double t, const orc_obstacle* obs, int n_obs, const orc_params* p);

double orc_rollout(const orc_problem* pr, const orc_params* p, uint32_t s, const double* eps,
                   double* useq, double* traj, double* alphas);
void orc_rollout_samples(const orc_problem* pr, const orc_params* p, const uint32_t* ids, int n,
                         int nthreads, double* J, double* useq);

int orc_weights(const double* J, int S, double lambda, double* wbar, double* m_out, double* Z_out);
int orc_solve(const orc_problem* pr, const orc_params* p, int nthreads, const double* eps,
              double* U_new, double* J, double* wbar, double* useq_all, double* stats);

void orc_plant_step(const double x[8], const double U0[3], const orc_params* p, double xn[8]);

#ifdef __cplusplus
}
#endif
#endif
