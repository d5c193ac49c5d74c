/*
 * mpm_oracle.c -- plain FP64 single-threaded CPU reference of one MLS-MPM
 * substep and its hand-derived reverse pass (ChainQueen, arXiv 1810.01054).
 *
 * TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and bench.py's
 * cpu_baseline leg load this library; the product path never does.
 *
 * Every loop runs in a fixed order: particles in index order, stencil
 * offsets lexicographic with the last axis fastest, grid nodes in storage
 * order.  Built with -O2 -ffp-contract=off (no FMA contraction, no
 * fast-math).  Nothing here is blocked, fused or reordered beyond the
 * equations it follows; each function names the passage it implements.
 *
 * Readings of the paper that this file relies on (the paper is silent or
 * garbled there):
 *   - constitutive model: compressible neo-Hookean,
 *       psi = mu/2 (tr F^T F - d) - mu ln J + la/2 (ln J)^2,
 *       P   = mu (F - F^-T) + la ln J F^-T;
 *   - node i sits at i*dx with dx = 1/n; stencil base = floor(x/dx - 0.5);
 *   - grid operations, in order: v^ = p/m (only where m > 0, else 0),
 *     v = v^ + dt g, then the boundary condition on wall nodes (any index
 *     < wall or >= n-wall; the paper omits gravity and boundaries in its
 *     main text): bc = 0 sets v = 0 (sticky walls); bc = 1 applies the
 *     friction projection of the supplement's section on friction
 *     projection gradients, (L), once per axis whose wall band holds the
 *     node, in axis order, low face before high face, with the inward
 *     normal of that face (+e_a at the low face, -e_a at the high face),
 *     friction coefficient c = s->friction and epsilon = 1e-12 in
 *     l_t = sqrt(|v_t|^2 + epsilon) (the paper gives no value);
 *   - actuation: sigma_pa = s_j * diag(axis) for the particle's actuator j;
 *     the total first Piola-Kirchhoff stress is P(F) + F sigma_pa;
 *   - in adjoint (J) the derivative of N is taken with respect to the
 *     particle position x_p (the printed derivative with respect to the node
 *     position would flip the sign of every such term);
 *   - in (E) the velocity multiplying dL/dv_i is the normalised momentum
 *     p_i/m_i before gravity is added;
 *   - per-particle materials (the paper's co-design and system
 *     identification): E_p and rho_p replace the scene's E and rho for
 *     particle p (nu and V0 stay per scene), m_p = rho_p V0.
 */
#include "mpm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* small dense helpers (row-major d x d)                               */
/* ------------------------------------------------------------------ */

static double det_d(int d, const double *A) {
  if (d == 2) return A[0] * A[3] - A[1] * A[2];
  return A[0] * (A[4] * A[8] - A[5] * A[7]) -
         A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* A^{-T} = cofactor(A) / det(A). */
static void inv_transpose_d(int d, const double *A, double J, double *R) {
  if (d == 2) {
    R[0] = A[3] / J;
    R[1] = -A[2] / J;
    R[2] = -A[1] / J;
    R[3] = A[0] / J;
    return;
  }
  R[0] = (A[4] * A[8] - A[5] * A[7]) / J;
  R[1] = -(A[3] * A[8] - A[5] * A[6]) / J;
  R[2] = (A[3] * A[7] - A[4] * A[6]) / J;
  R[3] = -(A[1] * A[8] - A[2] * A[7]) / J;
  R[4] = (A[0] * A[8] - A[2] * A[6]) / J;
  R[5] = -(A[0] * A[7] - A[1] * A[6]) / J;
  R[6] = (A[1] * A[5] - A[2] * A[4]) / J;
  R[7] = -(A[0] * A[5] - A[2] * A[3]) / J;
  R[8] = (A[0] * A[4] - A[1] * A[3]) / J;
}

/* R = A B (d x d). */
static void matmul_d(int d, const double *A, const double *B, double *R) {
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double s = 0.0;
      for (int g = 0; g < d; ++g) s += A[a * d + g] * B[g * d + b];
      R[a * d + b] = s;
    }
}

/* R = A^T B (d x d). */
static void matmul_tn_d(int d, const double *A, const double *B, double *R) {
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double s = 0.0;
      for (int g = 0; g < d; ++g) s += A[g * d + a] * B[g * d + b];
      R[a * d + b] = s;
    }
}

/* R = A B^T (d x d). */
static void matmul_nt_d(int d, const double *A, const double *B, double *R) {
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double s = 0.0;
      for (int g = 0; g < d; ++g) s += A[a * d + g] * B[b * d + g];
      R[a * d + b] = s;
    }
}

static int all_finite(const double *a, int n) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(a[i])) return 0;
  return 1;
}

/* ------------------------------------------------------------------ */
/* material model (Table I: P = dpsi/dF; supplement: hyperelastic with  */
/* E_p, nu_p)                                                           */
/* ------------------------------------------------------------------ */

void orc_lame(double E, double nu, double *mu, double *la) {
  *mu = E / (2.0 * (1.0 + nu));
  *la = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
}

int orc_neohookean_P(int d, double mu, double la, const double *F, double *P) {
  double J = det_d(d, F);
  if (!isfinite(J)) return ORC_ERR_NONFINITE;
  if (J <= 0.0) return ORC_ERR_INVERTED;
  double FiT[9];
  inv_transpose_d(d, F, J, FiT);
  double lnJ = log(J);
  for (int k = 0; k < d * d; ++k)
    P[k] = mu * (F[k] - FiT[k]) + la * lnJ * FiT[k];
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* quadratic B-spline (Table I: N; the affine scale D = 4/dx^2)         */
/* ------------------------------------------------------------------ */

/* N(u) for u = (x_p - x_i)/dx, and dN/du. */
static double bspline_N(double u) {
  double a = fabs(u);
  if (a < 0.5) return 0.75 - u * u;
  if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
  return 0.0;
}

static double bspline_dN(double u) {
  double a = fabs(u);
  if (a < 0.5) return -2.0 * u;
  if (a < 1.5) return (u > 0.0 ? -1.0 : 1.0) * (1.5 - a);
  return 0.0;
}

void orc_bspline(double xp, double inv_dx, int32_t *base, double *fx,
                 double w[3], double dw[3]) {
  double dx = 1.0 / inv_dx;
  int32_t b = (int32_t)floor(xp * inv_dx - 0.5);
  *base = b;
  *fx = xp * inv_dx - (double)b;
  for (int k = 0; k < 3; ++k) {
    double u = (xp - (double)(b + k) * dx) * inv_dx;
    w[k] = bspline_N(u);
    dw[k] = bspline_dN(u) * inv_dx; /* d/dx_p of N((x_p - x_i)/dx) */
  }
}

/* ------------------------------------------------------------------ */
/* per-particle stencil                                                 */
/* ------------------------------------------------------------------ */

typedef struct stencil {
  int d, n;
  int32_t base[3];
  double w[3][3], dw[3][3];
} stencil;

static int stencil_setup(const orc_scene *s, const double *xp, stencil *st) {
  int d = s->dim, n = s->n_grid;
  double inv_dx = (double)n;
  st->d = d;
  st->n = n;
  for (int a = 0; a < d; ++a) {
    if (!isfinite(xp[a])) return ORC_ERR_NONFINITE;
    double xs = xp[a] * inv_dx - 0.5;
    if (xs < -1.0 || xs > (double)n) return ORC_ERR_DOMAIN;
    double fx;
    orc_bspline(xp[a], inv_dx, &st->base[a], &fx, st->w[a], st->dw[a]);
    if (st->base[a] < 0 || st->base[a] > n - 3) return ORC_ERR_DOMAIN;
  }
  return ORC_OK;
}

static int n_stencil(int d) { return d == 2 ? 9 : 27; }

/* Offset o (last axis fastest) -> per-axis offsets. */
static void stencil_offsets(int d, int o, int off[3]) {
  if (d == 2) {
    off[0] = o / 3;
    off[1] = o % 3;
    off[2] = 0;
  } else {
    off[0] = o / 9;
    off[1] = (o / 3) % 3;
    off[2] = o % 3;
  }
}

static long node_index(const stencil *st, const int off[3]) {
  long i = st->base[0] + off[0];
  for (int a = 1; a < st->d; ++a) i = i * st->n + (st->base[a] + off[a]);
  return i;
}

/* Weight N, its gradient w.r.t. x_p, and delta = x_i - x_p. */
static double stencil_weight(const stencil *st, const double *xp,
                             const int off[3], double gradN[3],
                             double delta[3]) {
  int d = st->d;
  double dx = 1.0 / (double)st->n;
  double N = 1.0;
  for (int a = 0; a < d; ++a) N *= st->w[a][off[a]];
  for (int a = 0; a < d; ++a) {
    double g = st->dw[a][off[a]];
    for (int b = 0; b < d; ++b)
      if (b != a) g *= st->w[b][off[b]];
    gradN[a] = g;
    delta[a] = (double)(st->base[a] + off[a]) * dx - xp[a];
  }
  return N;
}

static long n_nodes(const orc_scene *s) {
  long n = s->n_grid;
  return s->dim == 2 ? n * n : n * n * n;
}

static void load_particle(const orc_scene *s, long p, const double *x,
                          const double *v, const double *C, const double *F,
                          double xp[3], double vp[3], double Cp[9],
                          double Fp[9]) {
  int d = s->dim;
  long N = s->n_particles;
  for (int a = 0; a < d; ++a) {
    if (x) xp[a] = x[a * N + p];
    if (v) vp[a] = v[a * N + p];
  }
  for (int k = 0; k < d * d; ++k) {
    if (C) Cp[k] = C[k * N + p];
    if (F) Fp[k] = F[k * N + p];
  }
}

static int scene_ok(const orc_scene *s) {
  if (!s) return 0;
  if (s->dim != 2 && s->dim != 3) return 0;
  if (s->n_grid < 3 || s->n_particles < 0 || s->n_act < 0 || s->wall < 0)
    return 0;
  if (s->bc != 0 && s->bc != 1) return 0;
  if (s->bc == 1 && !(s->friction >= 0.0)) return 0;
  return 1;
}

/* Per-particle stress quantities: P (elastic), Pt = P + F sigma, G. */
typedef struct stress {
  double P[9], Pt[9], G[9], FiT[9], sigma[3];
  double J, lnJ;
} stress;

/* Material of particle p: Lame parameters from E_p (or the scene's E) and
 * the scene's nu; mass m_p = rho_p V0 (or the scene's rho). */
static void particle_material(const orc_scene *s, long p, double *mu, double *la,
                              double *mp) {
  orc_lame(s->E_p ? s->E_p[p] : s->E, s->nu, mu, la);
  *mp = (s->rho_p ? s->rho_p[p] : s->rho) * s->V0;
}

static int particle_stress(const orc_scene *s, const int32_t *act_id,
                           const double *act, long p, const double *Cp,
                           const double *Fp, stress *out) {
  int d = s->dim;
  double mu, la, mp;
  particle_material(s, p, &mu, &la, &mp);
  double dx = 1.0 / (double)s->n_grid;
  double Dinv = 4.0 / (dx * dx);
  int rc = orc_neohookean_P(d, mu, la, Fp, out->P);
  if (rc) return rc;
  out->J = det_d(d, Fp);
  out->lnJ = log(out->J);
  inv_transpose_d(d, Fp, out->J, out->FiT);
  int j = act_id ? act_id[p] : -1;
  for (int b = 0; b < d; ++b)
    out->sigma[b] = (j >= 0) ? act[j] * s->act_axis[b] : 0.0;
  /* P_p^n = P(F_p^n) + F_p sigma_pa  (section III, actuation model) */
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b)
      out->Pt[a * d + b] = out->P[a * d + b] + Fp[a * d + b] * out->sigma[b];
  /* G_p = -(4/dx^2) dt V_p^0 P_p F_p^T + m_p C_p  (section III, P2G) */
  double PFt[9];
  matmul_nt_d(d, out->Pt, Fp, PFt);
  for (int k = 0; k < d * d; ++k)
    out->G[k] = -Dinv * s->dt * s->V0 * PFt[k] + mp * Cp[k];
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* forward: section III, steps 1-3                                      */
/* ------------------------------------------------------------------ */

int orc_p2g(const orc_scene *s, const int32_t *act_id, const double *act,
            const double *x, const double *v, const double *C, const double *F,
            double *gm, double *gp) {
  if (!scene_ok(s)) return ORC_ERR_ARG;
  int d = s->dim;
  long nn = n_nodes(s);
  memset(gm, 0, sizeof(double) * nn);
  memset(gp, 0, sizeof(double) * nn * d);
  for (long p = 0; p < s->n_particles; ++p) {
    double xp[3], vp[3], Cp[9], Fp[9], mu, la, mp;
    particle_material(s, p, &mu, &la, &mp);
    load_particle(s, p, x, v, C, F, xp, vp, Cp, Fp);
    stencil st;
    int rc = stencil_setup(s, xp, &st);
    if (rc) return rc;
    stress sp;
    rc = particle_stress(s, act_id, act, p, Cp, Fp, &sp);
    if (rc) return rc;
    for (int o = 0; o < n_stencil(d); ++o) {
      int off[3];
      double gradN[3], delta[3];
      stencil_offsets(d, o, off);
      double N = stencil_weight(&st, xp, off, gradN, delta);
      long i = node_index(&st, off);
      /* m_i = sum_p N m_p */
      gm[i] += N * mp;
      /* p_i = sum_p N [m_p v_p + G_p (x_i - x_p)] */
      for (int a = 0; a < d; ++a) {
        double Gd = 0.0;
        for (int b = 0; b < d; ++b) Gd += sp.G[a * d + b] * delta[b];
        gp[a * nn + i] += N * (mp * vp[a] + Gd);
      }
    }
  }
  return ORC_OK;
}

static int is_wall_node(const orc_scene *s, long i) {
  int n = s->n_grid, d = s->dim;
  for (int a = d - 1; a >= 0; --a) {
    int ia = (int)(i % n);
    i /= n;
    if (ia < s->wall || ia >= n - s->wall) return 1;
  }
  return 0;
}

/* (L) forward: friction projection of the node velocity v against a wall
 * with unit normal nrm and friction coefficient c:
 *   l_n = v . n,  v_t = v - l_n n,  l_t = sqrt(|v_t|^2 + eps),
 *   v^_t = v_t / l_t,  l*_t = max(l_t + c min(l_n, 0), 0),
 *   v* = l*_t v^_t + max(l_n, 0) n. */
#define ORC_FRICTION_EPS 1e-12
void orc_friction_project(int d, const double *nrm, double c, const double *v,
                          double *vs) {
  double ln = 0.0;
  for (int a = 0; a < d; ++a) ln += v[a] * nrm[a];
  double vt[3], lt2 = 0.0;
  for (int a = 0; a < d; ++a) {
    vt[a] = v[a] - ln * nrm[a];
    lt2 += vt[a] * vt[a];
  }
  double lt = sqrt(lt2 + ORC_FRICTION_EPS);
  double lts = fmax(lt + c * fmin(ln, 0.0), 0.0);
  for (int a = 0; a < d; ++a) vs[a] = lts * (vt[a] / lt) + fmax(ln, 0.0) * nrm[a];
}

/* (L) reverse: dL/dv (vb) from dL/dv* (vbs) at the same v, with
 * H(x) = [x >= 0] and R = l_t + c min(l_n, 0). */
void orc_friction_project_bwd(int d, const double *nrm, double c,
                              const double *v, const double *vbs, double *vb) {
  double ln = 0.0;
  for (int a = 0; a < d; ++a) ln += v[a] * nrm[a];
  double vt[3], lt2 = 0.0;
  for (int a = 0; a < d; ++a) {
    vt[a] = v[a] - ln * nrm[a];
    lt2 += vt[a] * vt[a];
  }
  double lt = sqrt(lt2 + ORC_FRICTION_EPS);
  double vth[3];
  for (int a = 0; a < d; ++a) vth[a] = vt[a] / lt;
  double R = lt + c * fmin(ln, 0.0);
  double lts = fmax(R, 0.0);
  double HR = R >= 0.0 ? 1.0 : 0.0;
  /* dL/dl*_t and dL/dv^_t */
  double ltsb = 0.0, vthb[3];
  for (int a = 0; a < d; ++a) {
    ltsb += vbs[a] * vth[a];
    vthb[a] = vbs[a] * lts;
  }
  /* dL/dl_t */
  double s = 0.0;
  for (int a = 0; a < d; ++a) s += vt[a] * vthb[a];
  double ltb = -s / (lt * lt) + ltsb * HR;
  /* dL/dv_t */
  double vtb[3];
  for (int a = 0; a < d; ++a) vtb[a] = (ltb * vt[a] + vthb[a]) / lt;
  /* dL/dl_n */
  double lnb = 0.0, nv = 0.0;
  for (int a = 0; a < d; ++a) {
    lnb -= vtb[a] * nrm[a];
    nv += nrm[a] * vbs[a];
  }
  lnb += ltsb * HR * c * (-ln >= 0.0 ? 1.0 : 0.0);
  lnb += (ln >= 0.0 ? 1.0 : 0.0) * nv;
  for (int a = 0; a < d; ++a) vb[a] = lnb * nrm[a] + vtb[a];
}

/* The boundary faces of node i in the order the projection visits them
 * (axis order, low face before high face): their count, and the inward
 * normal of each (stage k: axis ax[k], sign sg[k]). */
static int wall_faces(const orc_scene *s, long i, int *ax, double *sg) {
  int n = s->n_grid, d = s->dim, idx[3], k = 0;
  for (int a = d - 1; a >= 0; --a) {
    idx[a] = (int)(i % n);
    i /= n;
  }
  for (int a = 0; a < d; ++a) {
    if (idx[a] < s->wall) {
      ax[k] = a;
      sg[k++] = 1.0;
    }
    if (idx[a] >= n - s->wall) {
      ax[k] = a;
      sg[k++] = -1.0;
    }
  }
  return k;
}

/* Boundary condition on one wall node: v (in place). */
static void wall_bc(const orc_scene *s, long i, double *v) {
  if (s->bc == 0) {
    for (int a = 0; a < s->dim; ++a) v[a] = 0.0;
    return;
  }
  int ax[6];
  double sg[6];
  int nf = wall_faces(s, i, ax, sg);
  for (int k = 0; k < nf; ++k) {
    double nrm[3] = {0.0, 0.0, 0.0}, out[3];
    nrm[ax[k]] = sg[k];
    orc_friction_project(s->dim, nrm, s->friction, v, out);
    for (int a = 0; a < s->dim; ++a) v[a] = out[a];
  }
}

/* Reverse of wall_bc: vb (dL/dv after the condition) -> dL/dv before it,
 * in place; v is the velocity before the condition. */
static void wall_bc_bwd(const orc_scene *s, long i, const double *v, double *vb) {
  if (s->bc == 0) {
    for (int a = 0; a < s->dim; ++a) vb[a] = 0.0;
    return;
  }
  int ax[6];
  double sg[6], vin[7][3];
  int nf = wall_faces(s, i, ax, sg);
  for (int a = 0; a < s->dim; ++a) vin[0][a] = v[a];
  for (int k = 0; k < nf; ++k) {
    double nrm[3] = {0.0, 0.0, 0.0};
    nrm[ax[k]] = sg[k];
    orc_friction_project(s->dim, nrm, s->friction, vin[k], vin[k + 1]);
  }
  for (int k = nf - 1; k >= 0; --k) {
    double nrm[3] = {0.0, 0.0, 0.0}, out[3];
    nrm[ax[k]] = sg[k];
    orc_friction_project_bwd(s->dim, nrm, s->friction, vin[k], vb, out);
    for (int a = 0; a < s->dim; ++a) vb[a] = out[a];
  }
}

int orc_grid_update(const orc_scene *s, const double *gm, const double *gp,
                    double *gv) {
  if (!scene_ok(s)) return ORC_ERR_ARG;
  int d = s->dim;
  long nn = n_nodes(s);
  for (long i = 0; i < nn; ++i) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d; ++a) {
      if (gm[i] > 0.0) {
        /* v_i = p_i / m_i, then gravity */
        v[a] = gp[a * nn + i] / gm[i];
        v[a] = v[a] + s->dt * s->gravity[a];
      }
    }
    if (is_wall_node(s, i)) wall_bc(s, i, v);
    for (int a = 0; a < d; ++a) gv[a * nn + i] = v[a];
  }
  return ORC_OK;
}

int orc_g2p(const orc_scene *s, const double *gv, const double *x,
            const double *F, double *x1, double *v1, double *C1, double *F1) {
  if (!scene_ok(s)) return ORC_ERR_ARG;
  int d = s->dim;
  long N = s->n_particles, nn = n_nodes(s);
  double dx = 1.0 / (double)s->n_grid;
  double Dinv = 4.0 / (dx * dx);
  for (long p = 0; p < N; ++p) {
    double xp[3], Fp[9];
    load_particle(s, p, x, NULL, NULL, F, xp, NULL, NULL, Fp);
    stencil st;
    int rc = stencil_setup(s, xp, &st);
    if (rc) return rc;
    double vn[3] = {0, 0, 0}, B[9] = {0};
    for (int o = 0; o < n_stencil(d); ++o) {
      int off[3];
      double gradN[3], delta[3];
      stencil_offsets(d, o, off);
      double Nw = stencil_weight(&st, xp, off, gradN, delta);
      long i = node_index(&st, off);
      for (int a = 0; a < d; ++a) {
        double via = gv[a * nn + i];
        /* v_p^{n+1} = sum_i N v_i */
        vn[a] += Nw * via;
        /* C_p^{n+1} = (4/dx^2) sum_i N v_i (x_i - x_p)^T */
        for (int b = 0; b < d; ++b) B[a * d + b] += Nw * via * delta[b];
      }
    }
    double Cn[9], Fn[9], Ipc[9];
    for (int k = 0; k < d * d; ++k) Cn[k] = Dinv * B[k];
    /* F_p^{n+1} = (I + dt C_p^{n+1}) F_p^n */
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b)
        Ipc[a * d + b] = (a == b ? 1.0 : 0.0) + s->dt * Cn[a * d + b];
    matmul_d(d, Ipc, Fp, Fn);
    double xn[3];
    /* x_p^{n+1} = x_p^n + dt v_p^{n+1} */
    for (int a = 0; a < d; ++a) xn[a] = xp[a] + s->dt * vn[a];
    if (!all_finite(vn, d) || !all_finite(xn, d) || !all_finite(Cn, d * d) ||
        !all_finite(Fn, d * d))
      return ORC_ERR_NONFINITE;
    for (int a = 0; a < d; ++a) {
      x1[a * N + p] = xn[a];
      v1[a * N + p] = vn[a];
    }
    for (int k = 0; k < d * d; ++k) {
      C1[k * N + p] = Cn[k];
      F1[k * N + p] = Fn[k];
    }
  }
  return ORC_OK;
}

int orc_step_fwd(const orc_scene *s, const int32_t *act_id, const double *act,
                 const double *x, const double *v, const double *C,
                 const double *F, double *x1, double *v1, double *C1,
                 double *F1) {
  if (!scene_ok(s)) return ORC_ERR_ARG;
  long nn = n_nodes(s);
  int d = s->dim;
  double *gm = (double *)malloc(sizeof(double) * nn);
  double *gp = (double *)malloc(sizeof(double) * nn * d);
  double *gv = (double *)malloc(sizeof(double) * nn * d);
  int rc = ORC_ERR_OOM;
  if (gm && gp && gv) {
    rc = orc_p2g(s, act_id, act, x, v, C, F, gm, gp);
    if (!rc) rc = orc_grid_update(s, gm, gp, gv);
    if (!rc) rc = orc_g2p(s, gv, x, F, x1, v1, C1, F1);
  }
  free(gm);
  free(gp);
  free(gv);
  return rc;
}

/* ------------------------------------------------------------------ */
/* reverse: supplement, backward P2G (A-C), backward grid (D-E),        */
/* backward G2P (F-K)                                                   */
/* ------------------------------------------------------------------ */

int orc_step_bwd(const orc_scene *s, const int32_t *act_id, const double *act,
                 const double *x, const double *v, const double *C,
                 const double *F, const double *gx1, const double *gv1,
                 const double *gC1, const double *gF1, double *gx, double *gv,
                 double *gC, double *gF, double *g_act) {
  if (!scene_ok(s)) return ORC_ERR_ARG;
  int d = s->dim, ns = n_stencil(d);
  long N = s->n_particles, nn = n_nodes(s);
  double dx = 1.0 / (double)s->n_grid;
  double Dinv = 4.0 / (dx * dx);
  double dt = s->dt;
  /* d mu / dE and d la / dE (Lame parameters are linear in E) */
  double dmu_dE, dla_dE;
  orc_lame(1.0, s->nu, &dmu_dE, &dla_dE);

  double *gm = (double *)malloc(sizeof(double) * nn);
  double *gpm = (double *)malloc(sizeof(double) * nn * d);
  double *gvel = (double *)malloc(sizeof(double) * nn * d);
  double *vbar = (double *)calloc((size_t)(nn * d), sizeof(double));
  double *pbar = (double *)malloc(sizeof(double) * nn * d);
  double *mbar = (double *)malloc(sizeof(double) * nn);
  int rc = ORC_ERR_OOM;
  if (!gm || !gpm || !gvel || !vbar || !pbar || !mbar) goto done;

  /* recompute the forward grid of this step */
  rc = orc_p2g(s, act_id, act, x, v, C, F, gm, gpm);
  if (rc) goto done;
  rc = orc_grid_update(s, gm, gpm, gvel);
  if (rc) goto done;

  /* R1 -- backward P2G: scatter particle adjoints to dL/dv_i. */
  for (long p = 0; p < N; ++p) {
    double xp[3], Fp[9], gx1p[3], gv1p[3], gC1p[9], gF1p[9];
    load_particle(s, p, x, NULL, NULL, F, xp, NULL, NULL, Fp);
    load_particle(s, p, gx1, gv1, gC1, gF1, gx1p, gv1p, gC1p, gF1p);
    stencil st;
    rc = stencil_setup(s, xp, &st);
    if (rc) goto done;
    /* (A) dL/dv_p^{n+1} = dt dL/dx_p^{n+1}, plus the carried dL/dv_p^{n+1}. */
    double vt[3];
    for (int a = 0; a < d; ++a) vt[a] = gv1p[a] + dt * gx1p[a];
    /* (B) dL/dC^{n+1} = dt dL/dF^{n+1} F^{nT}, plus the carried dL/dC. */
    double Ct[9], GFt[9];
    matmul_nt_d(d, gF1p, Fp, GFt);
    for (int k = 0; k < d * d; ++k) Ct[k] = gC1p[k] + dt * GFt[k];
    /* (C) dL/dv_i = sum_p N [vt + (4/dx^2) Ct (x_i - x_p)] */
    for (int o = 0; o < ns; ++o) {
      int off[3];
      double gradN[3], delta[3];
      stencil_offsets(d, o, off);
      double Nw = stencil_weight(&st, xp, off, gradN, delta);
      long i = node_index(&st, off);
      for (int a = 0; a < d; ++a) {
        double Cd = 0.0;
        for (int b = 0; b < d; ++b) Cd += Ct[a * d + b] * delta[b];
        vbar[a * nn + i] += Nw * (vt[a] + Dinv * Cd);
      }
    }
  }

  /* R2 -- backward grid operations. */
  for (long i = 0; i < nn; ++i) {
    int wall = is_wall_node(s, i);
    double m = gm[i];
    if ((wall && s->bc == 0) || !(m > 0.0)) {
      for (int a = 0; a < d; ++a) pbar[a * nn + i] = 0.0;
      mbar[i] = 0.0;
      continue;
    }
    /* dL/dv before the boundary condition: (L) on wall nodes */
    double vb[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d; ++a) vb[a] = vbar[a * nn + i];
    if (wall) {
      double v[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < d; ++a) v[a] = gpm[a * nn + i] / m + s->dt * s->gravity[a];
      wall_bc_bwd(s, i, v, vb);
    }
    double vdot = 0.0;
    for (int a = 0; a < d; ++a) {
      /* (D) dL/dp_i = dL/dv_i / m_i  (gravity passes dL/dv_i unchanged) */
      pbar[a * nn + i] = vb[a] / m;
      double vhat = gpm[a * nn + i] / m;
      vdot += vhat * vb[a];
    }
    /* (E) dL/dm_i = -(1/m_i) sum_a v^_ia dL/dv_ia, v^ = p/m before gravity */
    mbar[i] = -vdot / m;
  }

  /* R3 -- backward G2P: gather grid adjoints to particle adjoints. */
  for (long p = 0; p < N; ++p) {
    double xp[3], vp[3], Cp[9], Fp[9], gx1p[3], gv1p[3], gC1p[9], gF1p[9];
    load_particle(s, p, x, v, C, F, xp, vp, Cp, Fp);
    load_particle(s, p, gx1, gv1, gC1, gF1, gx1p, gv1p, gC1p, gF1p);
    stencil st;
    rc = stencil_setup(s, xp, &st);
    if (rc) goto done;
    stress sp;
    rc = particle_stress(s, act_id, act, p, Cp, Fp, &sp);
    if (rc) goto done;
    double mu, la, mp;
    particle_material(s, p, &mu, &la, &mp);

    /* C_p^{n+1}, recomputed as in the forward G2P */
    double B[9] = {0};
    for (int o = 0; o < ns; ++o) {
      int off[3];
      double gradN[3], delta[3];
      stencil_offsets(d, o, off);
      double Nw = stencil_weight(&st, xp, off, gradN, delta);
      long i = node_index(&st, off);
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b)
          B[a * d + b] += Nw * gvel[a * nn + i] * delta[b];
    }
    double C1p[9];
    for (int k = 0; k < d * d; ++k) C1p[k] = Dinv * B[k];

    double vt[3], Ct[9], GFt[9];
    for (int a = 0; a < d; ++a) vt[a] = gv1p[a] + dt * gx1p[a];
    matmul_nt_d(d, gF1p, Fp, GFt);
    for (int k = 0; k < d * d; ++k) Ct[k] = gC1p[k] + dt * GFt[k];

    double xb[3], vb[3] = {0, 0, 0}, Gb[9] = {0};
    double Spb[3] = {0, 0, 0}, Nmb = 0.0;  /* sum N dL/dp_i, sum N dL/dm_i */
    /* x_p^{n+1} = x_p^n + dt v^{n+1}: the direct term of (J) */
    for (int a = 0; a < d; ++a) xb[a] = gx1p[a];

    for (int o = 0; o < ns; ++o) {
      int off[3];
      double gradN[3], delta[3];
      stencil_offsets(d, o, off);
      double Nw = stencil_weight(&st, xp, off, gradN, delta);
      long i = node_index(&st, off);
      double pb[3], vi[3], mb = mbar[i];
      for (int a = 0; a < d; ++a) {
        pb[a] = pbar[a * nn + i];
        vi[a] = gvel[a * nn + i];
      }
      for (int a = 0; a < d; ++a) {
        /* (F) dL/dv_p^n += N m_p dL/dp_i */
        vb[a] += Nw * mp * pb[a];
        Spb[a] += Nw * pb[a];
        /* dL/dG_p += N dL/dp_i (x_i - x_p)^T, used by (G), (H), (I) */
        for (int b = 0; b < d; ++b) Gb[a * d + b] += Nw * pb[a] * delta[b];
      }
      /* (J): scalar factors multiplying dN/dx_p */
      double s_v = 0.0, s_C = 0.0, s_p = 0.0;
      for (int a = 0; a < d; ++a) {
        s_v += vt[a] * vi[a];
        double Cd = 0.0, q = mp * vp[a];
        for (int b = 0; b < d; ++b) {
          Cd += Ct[a * d + b] * delta[b];
          q += sp.G[a * d + b] * delta[b];
        }
        s_C += vi[a] * Cd;
        s_p += pb[a] * q;
      }
      double s_all = s_v + Dinv * s_C + s_p + mp * mb;
      Nmb += Nw * mb;
      for (int c = 0; c < d; ++c) {
        /* (J): dN/dx_p terms of v^{n+1}, C^{n+1}, p_i and m_i */
        xb[c] += gradN[c] * s_all;
        /* (J): d(x_i - x_p)/dx_p = -I terms of C^{n+1} and p_i */
        double cterm = 0.0, pterm = 0.0;
        for (int a = 0; a < d; ++a) {
          cterm += vi[a] * Ct[a * d + c];
          pterm += pb[a] * sp.G[a * d + c];
        }
        xb[c] += -Nw * Dinv * cterm - Nw * pterm;
      }
    }

    /* (I) dL/dC_p^n = m_p dL/dG */
    double Cb[9];
    for (int k = 0; k < d * d; ++k) Cb[k] = mp * Gb[k];
    /* (G) dL/dP_p^n = -(4/dx^2) dt V^0 dL/dG F_p^n */
    double kG = -Dinv * dt * s->V0;
    double GbF[9], Ptb[9];
    matmul_d(d, Gb, Fp, GbF);
    for (int k = 0; k < d * d; ++k) Ptb[k] = kG * GbF[k];

    /* (H) dL/dF_p^n, four terms */
    double Fb[9], Ipc[9], T1[9], T2[9];
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b)
        Ipc[a * d + b] = (a == b ? 1.0 : 0.0) + dt * C1p[a * d + b];
    matmul_tn_d(d, Ipc, gF1p, Fb);   /* (I + dt C^{n+1})^T dL/dF^{n+1} */
    matmul_tn_d(d, Gb, sp.Pt, T1);   /* dL/dG^T P_p (from G = k P F^T) */
    for (int k = 0; k < d * d; ++k) Fb[k] += kG * T1[k];
    for (int a = 0; a < d; ++a)      /* dL/dP sigma^T (actuation) */
      for (int b = 0; b < d; ++b) Fb[a * d + b] += Ptb[a * d + b] * sp.sigma[b];
    /* elastic Hessian term: adjoint of dP for P = mu (F - F^-T) + la lnJ F^-T
     *   mu Pb + (mu - la lnJ) F^-T Pb^T F^-T + la <Pb, F^-T> F^-T          */
    double PbT[9], tmp[9];
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) PbT[a * d + b] = Ptb[b * d + a];
    matmul_d(d, sp.FiT, PbT, tmp);
    matmul_d(d, tmp, sp.FiT, T2);
    double inner = 0.0;
    for (int k = 0; k < d * d; ++k) inner += Ptb[k] * sp.FiT[k];
    for (int k = 0; k < d * d; ++k)
      Fb[k] += mu * Ptb[k] + (mu - la * sp.lnJ) * T2[k] + la * inner * sp.FiT[k];

    /* per-particle materials (co-design, system identification):
     *   dL/dm_p = sum_i N [dL/dm_i + dL/dp_i . (v_p + C_p (x_i - x_p))]
     *           (m_p enters m_i, m_p v_p and G_p = ... + m_p C_p),
     *   dL/dmu_p = <dL/dP, F - F^-T>,  dL/dla_p = <dL/dP, ln J F^-T>,
     *   dL/dE_p = dL/dmu dmu/dE + dL/dla dla/dE,  dL/drho_p = V0 dL/dm_p */
    if (s->gE_p) {
      double mub = 0.0;
      for (int k = 0; k < d * d; ++k) mub += Ptb[k] * (Fp[k] - sp.FiT[k]);
      s->gE_p[p] += mub * dmu_dE + sp.lnJ * inner * dla_dE;
    }
    if (s->grho_p) {
      double mbp = Nmb;
      for (int a = 0; a < d; ++a) mbp += vp[a] * Spb[a];
      for (int k = 0; k < d * d; ++k) mbp += Cp[k] * Gb[k];
      s->grho_p[p] += s->V0 * mbp;
    }

    /* (K) dL/dsigma = F^T dL/dP; sigma = s_j diag(axis) */
    int j = act_id ? act_id[p] : -1;
    if (j >= 0 && g_act) {
      double sb = 0.0;
      for (int a = 0; a < d; ++a) {
        double sig_aa = 0.0;
        for (int g = 0; g < d; ++g) sig_aa += Fp[g * d + a] * Ptb[g * d + a];
        sb += s->act_axis[a] * sig_aa;
      }
      g_act[j] += sb;
    }

    if (!all_finite(xb, d) || !all_finite(vb, d) || !all_finite(Cb, d * d) ||
        !all_finite(Fb, d * d)) {
      rc = ORC_ERR_NONFINITE;
      goto done;
    }
    for (int a = 0; a < d; ++a) {
      gx[a * N + p] = xb[a];
      gv[a * N + p] = vb[a];
    }
    for (int k = 0; k < d * d; ++k) {
      gC[k * N + p] = Cb[k];
      gF[k * N + p] = Fb[k];
    }
  }
  rc = ORC_OK;

done:
  free(gm);
  free(gpm);
  free(gvel);
  free(vbar);
  free(pbar);
  free(mbar);
  return rc;
}

/* ------------------------------------------------------------------ */
/* rollouts: chain rule across steps over a memo of every state         */
/* (section III: states cached in a memo, gradients evaluated from it) */
/* ------------------------------------------------------------------ */

int orc_rollout(const orc_scene *s, const int32_t *act_id, int T,
                const double *act, const double *x0, const double *v0,
                const double *C0, const double *F0, double *xT, double *vT,
                double *CT, double *FT, const double *gxT, const double *gvT,
                const double *gCT, const double *gFT, double *gx0,
                double *gv0, double *gC0, double *gF0, double *g_act) {
  if (!scene_ok(s) || T < 0) return ORC_ERR_ARG;
  int d = s->dim, nact = s->n_act;
  long N = s->n_particles;
  size_t vs = (size_t)N * d, ms = (size_t)N * d * d;
  size_t ss = 2 * vs + 2 * ms; /* one state: x, v, C, F */
  double *memo = (double *)malloc(sizeof(double) * ss * (size_t)(T + 1) + 8);
  if (!memo) return ORC_ERR_OOM;
#define SX(n) (memo + (size_t)(n) * ss)
#define SV(n) (SX(n) + vs)
#define SC(n) (SX(n) + 2 * vs)
#define SF(n) (SX(n) + 2 * vs + ms)
  memcpy(SX(0), x0, sizeof(double) * vs);
  memcpy(SV(0), v0, sizeof(double) * vs);
  memcpy(SC(0), C0, sizeof(double) * ms);
  memcpy(SF(0), F0, sizeof(double) * ms);
  int rc = ORC_OK;
  for (int n = 0; n < T && !rc; ++n)
    rc = orc_step_fwd(s, act_id, act + (size_t)n * nact, SX(n), SV(n), SC(n),
                      SF(n), SX(n + 1), SV(n + 1), SC(n + 1), SF(n + 1));
  if (!rc) {
    memcpy(xT, SX(T), sizeof(double) * vs);
    memcpy(vT, SV(T), sizeof(double) * vs);
    memcpy(CT, SC(T), sizeof(double) * ms);
    memcpy(FT, SF(T), sizeof(double) * ms);
  }
  if (!rc && gxT) {
    double *a1 = (double *)malloc(sizeof(double) * ss + 8);
    double *a0 = (double *)malloc(sizeof(double) * ss + 8);
    if (!a1 || !a0) {
      rc = ORC_ERR_OOM;
    } else {
      memcpy(a1, gxT, sizeof(double) * vs);
      memcpy(a1 + vs, gvT, sizeof(double) * vs);
      memcpy(a1 + 2 * vs, gCT, sizeof(double) * ms);
      memcpy(a1 + 2 * vs + ms, gFT, sizeof(double) * ms);
      if (g_act) memset(g_act, 0, sizeof(double) * (size_t)T * nact);
      for (int n = T - 1; n >= 0 && !rc; --n) {
        rc = orc_step_bwd(s, act_id, act + (size_t)n * nact, SX(n), SV(n),
                          SC(n), SF(n), a1, a1 + vs, a1 + 2 * vs,
                          a1 + 2 * vs + ms, a0, a0 + vs, a0 + 2 * vs,
                          a0 + 2 * vs + ms,
                          g_act ? g_act + (size_t)n * nact : NULL);
        double *t = a0;
        a0 = a1;
        a1 = t;
      }
      if (!rc) {
        memcpy(gx0, a1, sizeof(double) * vs);
        memcpy(gv0, a1 + vs, sizeof(double) * vs);
        memcpy(gC0, a1 + 2 * vs, sizeof(double) * ms);
        memcpy(gF0, a1 + 2 * vs + ms, sizeof(double) * ms);
      }
    }
    free(a1);
    free(a0);
  }
#undef SX
#undef SV
#undef SC
#undef SF
  free(memo);
  return rc;
}

/* ------------------------------------------------------------------ */
/* closed-loop controller a = tanh(W z + b) (section IV, Control)        */
/* ------------------------------------------------------------------ */

/* z = [target, per component: mean x, mean v] of one state. */
static void ctrl_state_vector(const orc_scene *s, const int32_t *comp_id,
                              int n_comp, const long *count,
                              const double *target, const double *x,
                              const double *v, double *z) {
  int d = s->dim;
  long N = s->n_particles;
  int nz = d * (1 + 2 * n_comp);
  for (int i = 0; i < nz; ++i) z[i] = 0.0;
  for (int a = 0; a < d; ++a) z[a] = target[a];
  for (long p = 0; p < N; ++p) {
    int c = comp_id[p];
    if (c < 0) continue;
    for (int a = 0; a < d; ++a) {
      z[d + 2 * d * c + a] += x[(size_t)a * N + p];
      z[d + 2 * d * c + d + a] += v[(size_t)a * N + p];
    }
  }
  for (int c = 0; c < n_comp; ++c)
    for (int i = 0; i < 2 * d; ++i) z[d + 2 * d * c + i] /= (double)count[c];
}

int orc_rollout_ctrl(const orc_scene *s, const int32_t *act_id,
                     const int32_t *comp_id, int n_comp, const double *W,
                     const double *b, const double *target, int T,
                     const double *x0, const double *v0, const double *C0,
                     const double *F0, double *xT, double *vT, double *CT,
                     double *FT, double *acts, const double *gxT,
                     const double *gvT, const double *gCT, const double *gFT,
                     double *gx0, double *gv0, double *gC0, double *gF0,
                     double *gW, double *gb) {
  if (!scene_ok(s) || T < 0 || n_comp < 1 || s->n_act < 1 || !comp_id)
    return ORC_ERR_ARG;
  int d = s->dim, nact = s->n_act, nz = d * (1 + 2 * n_comp);
  long N = s->n_particles;
  long *count = (long *)calloc((size_t)n_comp, sizeof(long));
  if (!count) return ORC_ERR_OOM;
  for (long p = 0; p < N; ++p) {
    if (comp_id[p] >= n_comp) {
      free(count);
      return ORC_ERR_ARG;
    }
    if (comp_id[p] >= 0) count[comp_id[p]]++;
  }
  for (int c = 0; c < n_comp; ++c)
    if (count[c] == 0) {
      free(count);
      return ORC_ERR_ARG;
    }
  size_t vs = (size_t)N * d, ms = (size_t)N * d * d;
  size_t ss = 2 * vs + 2 * ms;
  double *memo = (double *)malloc(sizeof(double) * ss * (size_t)(T + 1) + 8);
  double *Z = (double *)malloc(sizeof(double) * (size_t)nz * (T + 1) + 8);
  double *A = (double *)malloc(sizeof(double) * (size_t)nact * (T + 1) + 8);
  if (!memo || !Z || !A) {
    free(memo), free(Z), free(A), free(count);
    return ORC_ERR_OOM;
  }
#define SX(n) (memo + (size_t)(n) * ss)
#define SV(n) (SX(n) + vs)
#define SC(n) (SX(n) + 2 * vs)
#define SF(n) (SX(n) + 2 * vs + ms)
  memcpy(SX(0), x0, sizeof(double) * vs);
  memcpy(SV(0), v0, sizeof(double) * vs);
  memcpy(SC(0), C0, sizeof(double) * ms);
  memcpy(SF(0), F0, sizeof(double) * ms);
  int rc = ORC_OK;
  for (int n = 0; n < T && !rc; ++n) {
    double *z = Z + (size_t)n * nz, *a = A + (size_t)n * nact;
    ctrl_state_vector(s, comp_id, n_comp, count, target, SX(n), SV(n), z);
    for (int j = 0; j < nact; ++j) {
      double pre = b[j];
      for (int i = 0; i < nz; ++i) pre += W[(size_t)j * nz + i] * z[i];
      a[j] = tanh(pre);
    }
    rc = orc_step_fwd(s, act_id, a, SX(n), SV(n), SC(n), SF(n), SX(n + 1),
                      SV(n + 1), SC(n + 1), SF(n + 1));
  }
  if (!rc) {
    memcpy(xT, SX(T), sizeof(double) * vs);
    memcpy(vT, SV(T), sizeof(double) * vs);
    memcpy(CT, SC(T), sizeof(double) * ms);
    memcpy(FT, SF(T), sizeof(double) * ms);
    if (acts) memcpy(acts, A, sizeof(double) * (size_t)nact * T);
  }
  if (!rc && gxT) {
    double *a1 = (double *)malloc(sizeof(double) * ss + 8);
    double *a0 = (double *)malloc(sizeof(double) * ss + 8);
    double *sb = (double *)malloc(sizeof(double) * nact + 8);
    double *zb = (double *)malloc(sizeof(double) * nz + 8);
    if (!a1 || !a0 || !sb || !zb) {
      rc = ORC_ERR_OOM;
    } else {
      memcpy(a1, gxT, sizeof(double) * vs);
      memcpy(a1 + vs, gvT, sizeof(double) * vs);
      memcpy(a1 + 2 * vs, gCT, sizeof(double) * ms);
      memcpy(a1 + 2 * vs + ms, gFT, sizeof(double) * ms);
      memset(gW, 0, sizeof(double) * (size_t)nact * nz);
      memset(gb, 0, sizeof(double) * nact);
      for (int n = T - 1; n >= 0 && !rc; --n) {
        const double *z = Z + (size_t)n * nz, *a = A + (size_t)n * nact;
        memset(sb, 0, sizeof(double) * nact);
        rc = orc_step_bwd(s, act_id, a, SX(n), SV(n), SC(n), SF(n), a1,
                          a1 + vs, a1 + 2 * vs, a1 + 2 * vs + ms, a0, a0 + vs,
                          a0 + 2 * vs, a0 + 2 * vs + ms, sb);
        /* a = tanh(W z + b): dL/dpre = dL/da (1 - a^2) */
        for (int i = 0; i < nz; ++i) zb[i] = 0.0;
        for (int j = 0; j < nact; ++j) {
          double g = sb[j] * (1.0 - a[j] * a[j]);
          gb[j] += g;
          for (int i = 0; i < nz; ++i) {
            gW[(size_t)j * nz + i] += g * z[i];
            zb[i] += W[(size_t)j * nz + i] * g;
          }
        }
        /* z's means: each particle of component c gets dL/dz / N_c */
        for (long p = 0; p < N; ++p) {
          int c = comp_id[p];
          if (c < 0) continue;
          for (int k = 0; k < d; ++k) {
            a0[(size_t)k * N + p] += zb[d + 2 * d * c + k] / (double)count[c];
            a0[vs + (size_t)k * N + p] += zb[d + 2 * d * c + d + k] / (double)count[c];
          }
        }
        double *t = a0;
        a0 = a1;
        a1 = t;
      }
      if (!rc) {
        memcpy(gx0, a1, sizeof(double) * vs);
        memcpy(gv0, a1 + vs, sizeof(double) * vs);
        memcpy(gC0, a1 + 2 * vs, sizeof(double) * ms);
        memcpy(gF0, a1 + 2 * vs + ms, sizeof(double) * ms);
      }
    }
    free(a1), free(a0), free(sb), free(zb);
  }
#undef SX
#undef SV
#undef SC
#undef SF
  free(memo), free(Z), free(A), free(count);
  return rc;
}

/* ------------------------------------------------------------------ */
/* sinusoid actuation bank and its reverse                              */
/* ------------------------------------------------------------------ */

static const double ORC_TWO_PI = 6.283185307179586476925286766559;

void orc_act_bank_fwd(int T, int n_act, int n_freq, double dt,
                      const double *freq, const double *amp,
                      const double *phase, double *act) {
  for (int n = 0; n < T; ++n) {
    double t = (double)n * dt;
    for (int j = 0; j < n_act; ++j) {
      double s = 0.0;
      for (int k = 0; k < n_freq; ++k)
        s += amp[j * n_freq + k] *
             sin(ORC_TWO_PI * freq[k] * t + phase[j * n_freq + k]);
      act[(size_t)n * n_act + j] = s;
    }
  }
}

void orc_act_bank_bwd(int T, int n_act, int n_freq, double dt,
                      const double *freq, const double *amp,
                      const double *phase, const double *g_act,
                      double *g_amp, double *g_phase) {
  for (int j = 0; j < n_act; ++j)
    for (int k = 0; k < n_freq; ++k) {
      double ga = 0.0, gp = 0.0;
      for (int n = 0; n < T; ++n) {
        double th = ORC_TWO_PI * freq[k] * ((double)n * dt) + phase[j * n_freq + k];
        double g = g_act[(size_t)n * n_act + j];
        ga += g * sin(th);
        gp += g * amp[j * n_freq + k] * cos(th);
      }
      g_amp[j * n_freq + k] = ga;
      g_phase[j * n_freq + k] = gp;
    }
}
