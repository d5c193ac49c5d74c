/*
 * mpm_oracle.h -- plain FP64 single-threaded CPU reference for one MLS-MPM
 * substep and its reverse (adjoint) pass, written from ChainQueen
 * (Hu et al., arXiv 1810.01054).
 *
 * TEST INFRASTRUCTURE.  This library exists only to check the HIP path.
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg load
 * it; the product library (libmpm) never includes, links or calls it, and
 * the two share no source.
 *
 * Layout (all arrays host memory, FP64, structure of arrays):
 *   x, v      : [d][N]      component a of particle p at a*N + p
 *   C, F      : [d*d][N]    entry (a,b) of particle p at (a*d + b)*N + p
 *   grid m    : [n^d]       node (i0,i1[,i2]) at ((i0*n)+i1)*n+i2 (last axis fastest)
 *   grid p, v : [d][n^d]
 *   act_id    : int32 [N]   actuator of each particle, -1 = passive
 *   act       : [n_act]     per-substep actuation scalars s_j (one step),
 *               [T][n_act]  for rollouts
 *
 * Return codes are 0 on success or one of the negative ORC_ERR_* values; the
 * first error met (in particle order) is returned and the outputs are then
 * unspecified.
 */
#ifndef MPM_ORACLE_H
#define MPM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_ERR_ARG = -1,
  ORC_ERR_OOM = -2,
  ORC_ERR_DOMAIN = -3,    /* a stencil base lies outside [0, n-3] */
  ORC_ERR_INVERTED = -4,  /* det F <= 0 */
  ORC_ERR_NONFINITE = -5  /* a non-finite value was produced */
};

typedef struct orc_scene {
  int32_t dim;         /* 2 or 3 */
  int32_t n_grid;      /* nodes per axis n; dx = 1/n, node i sits at i*dx */
  int32_t n_particles; /* N */
  int32_t n_act;       /* number of actuators */
  int32_t wall;        /* wall thickness in nodes */
  int32_t bc;          /* wall nodes: 0 sticky (v = 0), 1 friction projection (L) */
  double dt, E, nu, rho, V0; /* time step, Young's modulus, Poisson ratio,
                                density, initial particle volume */
  double gravity[3];
  double act_axis[3];  /* sigma_pa = s_j * diag(act_axis) */
  double friction;     /* friction coefficient c of (L), bc = 1 */
  /* per-particle materials (nullable [N]): E_p, rho_p replace E, rho for
   * particle p; the reverse pass ADDS dL/dE_p, dL/drho_p to gE_p, grho_p
   * (nullable [N]) */
  const double *E_p, *rho_p;
  double *gE_p, *grho_p;
} orc_scene;

/* (L) friction projection of one node velocity v (d entries) against a wall
 * with unit normal nrm and coefficient c (forward: vs = v*), and its reverse
 * (vb = dL/dv from vbs = dL/dv* at the same v). */
void orc_friction_project(int d, const double *nrm, double c, const double *v,
                          double *vs);
void orc_friction_project_bwd(int d, const double *nrm, double c,
                              const double *v, const double *vbs, double *vb);

/* Quadratic B-spline along one axis: stencil base, weights w[3] of the three
 * nodes base..base+2 and their derivatives dw[3] with respect to the particle
 * coordinate (not the node coordinate). */
void orc_bspline(double xp, double inv_dx, int32_t *base, double *fx,
                 double w[3], double dw[3]);

/* Compressible neo-Hookean first Piola-Kirchhoff stress P(F) (d x d,
 * row-major).  Returns ORC_ERR_INVERTED when det F <= 0. */
int orc_neohookean_P(int dim, double mu, double la, const double *F, double *P);

/* Lame parameters from (E, nu). */
void orc_lame(double E, double nu, double *mu, double *la);

/* Stage 1 (P2G): grid mass m[n^d] and momentum p[d][n^d] (both overwritten). */
int orc_p2g(const orc_scene *s, const int32_t *act_id, const double *act,
            const double *x, const double *v, const double *C, const double *F,
            double *gm, double *gp);

/* Stage 2 (grid operations): velocities v[d][n^d] from m and p, with gravity
 * and sticky walls. */
int orc_grid_update(const orc_scene *s, const double *gm, const double *gp,
                    double *gv);

/* Stage 3 (G2P): new particle state from the grid velocities. */
int orc_g2p(const orc_scene *s, const double *gv, const double *x,
            const double *F, double *x1, double *v1, double *C1, double *F1);

/* One full substep (stages 1-3). Outputs may not alias the inputs. */
int orc_step_fwd(const orc_scene *s, const int32_t *act_id, const double *act,
                 const double *x, const double *v, const double *C,
                 const double *F, double *x1, double *v1, double *C1,
                 double *F1);

/* Reverse of one substep: given state n and the adjoints of state n+1
 * (gx1, gv1, gC1, gF1), writes the adjoints of state n (gx, gv, gC, gF) and
 * ADDS dL/ds_j to g_act[j]. */
int orc_step_bwd(const orc_scene *s, const int32_t *act_id, const double *act,
                 const double *x, const double *v, const double *C,
                 const double *F, const double *gx1, const double *gv1,
                 const double *gC1, const double *gF1, double *gx, double *gv,
                 double *gC, double *gF, double *g_act);

/* T substeps from (x0,v0,C0,F0) with per-step actuation act[T][n_act]; the
 * final state goes to (xT,vT,CT,FT).  When gxT is non-NULL (then gvT, gCT,
 * gFT must be too) the reverse pass runs over a memo of every state and
 * writes the adjoints of the initial state (gx0,..) and g_act[T][n_act]
 * (overwritten). */
int orc_rollout(const orc_scene *s, const int32_t *act_id, int T,
                const double *act, const double *x0, const double *v0,
                const double *C0, const double *F0, double *xT, double *vT,
                double *CT, double *FT, const double *gxT, const double *gvT,
                const double *gCT, const double *gFT, double *gx0,
                double *gv0, double *gC0, double *gF0, double *g_act);

/* Closed-loop controller inside the rollout (section IV, Control): the
 * actuation of substep n is a^n = tanh(W z^n + b) with the state vector
 *   z^n = [target (d), then for each component c: the mean position and the
 *          mean velocity of its particles in state n (d each)],
 * nz = d (1 + 2 n_comp); comp_id[N] gives each particle's component (-1 =
 * none; every component must hold a particle).  W is [n_act][nz] row-major,
 * b [n_act], target [d].  Writes the final state and, if acts is non-NULL,
 * acts[T][n_act].  When gxT is non-NULL the memo reverse pass also writes
 * the adjoints of the initial state and dL/dW, dL/db (overwritten); the
 * controller's dependence on state n adds (dL/dz) / N_c to the position and
 * velocity adjoints of component c's particles. */
int orc_rollout_ctrl(const orc_scene *s, const int32_t *act_id,
                     const int32_t *comp_id, int n_comp, const double *W,
                     const double *b, const double *target, int T,
                     const double *x0, const double *v0, const double *C0,
                     const double *F0, double *xT, double *vT, double *CT,
                     double *FT, double *acts, const double *gxT,
                     const double *gvT, const double *gCT, const double *gFT,
                     double *gx0, double *gv0, double *gC0, double *gF0,
                     double *gW, double *gb);

/* Sinusoid actuation bank: act[n][j] = sum_k amp[j][k] sin(2 pi freq[k] t_n
 * + phase[j][k]) with t_n = n*dt. */
void orc_act_bank_fwd(int T, int n_act, int n_freq, double dt,
                      const double *freq, const double *amp,
                      const double *phase, double *act);
/* Its reverse: g_amp, g_phase [n_act][n_freq] (overwritten) from g_act. */
void orc_act_bank_bwd(int T, int n_act, int n_freq, double dt,
                      const double *freq, const double *amp,
                      const double *phase, const double *g_act,
                      double *g_amp, double *g_phase);

#ifdef __cplusplus
}
#endif
#endif
