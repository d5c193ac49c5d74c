/*
 * mpm.h -- C ABI of libmpm, an MI355X (gfx950) implementation of the
 * differentiable MLS-MPM substep of ChainQueen (Hu et al., arXiv 1810.01054):
 * particle-to-grid transfer, grid operations and grid-to-particle transfer
 * (section III, steps 1-3) and their reverse pass (supplement: backward P2G
 * (A)-(C), backward grid operations (D)-(E), backward G2P (F)-(K)).
 *
 * Conventions shared by every call
 * --------------------------------
 * Pointers marked DEVICE are device (HBM) addresses owned by the caller; the
 * library reads/writes them only during the call's stream-ordered work and
 * never frees or keeps them.  Pointers marked HOST are host memory, read
 * during the call only.  All floating-point data are FP32.
 *
 * A context holds one or more scenes of the same dimension d (2 or 3).  The
 * particles of all scenes are concatenated: scene s owns particles
 * [off_s, off_s + N_s) with off_s = N_0 + ... + N_{s-1}; N_tot is the total.
 * A particle state (Table I: x_p, v_p, C_p, F_p) is four DEVICE arrays in
 * structure-of-arrays layout:
 *     x, v : [d][N_tot]     component a of particle p at a*N_tot + p
 *     C, F : [d*d][N_tot]   entry (a,b) of particle p at (a*d+b)*N_tot + p
 * The adjoint of a state (dL/dx, dL/dv, dL/dC, dL/dF) uses the same struct
 * and layout.  Actuators are numbered per scene; actuator j of scene s has
 * the global index act_off_s + j with act_off_s = n_act_0 + ... + n_act_{s-1};
 * n_act_tot is the total.  Per-step actuation scalars s_j (the sigma_pa =
 * s_j diag(axis) of the actuation model) are FP32 [n_act_tot] per step.
 *
 * Grids are library-owned: scene s has n_s^d nodes at x_i = i/n_s, node
 * (i0,i1[,i2]) at linear index ((i0*n)+i1)*n+i2 (last axis fastest).
 *
 * Every call is asynchronous on the context's stream unless stated
 * otherwise.  Errors: calls return 0 (MPM_OK) or a negative MPM_ERR_* code.
 * Argument errors are detected on the host before any work is queued.
 * Errors detected by the kernels (MPM_ERR_DOMAIN, MPM_ERR_INVERTED,
 * MPM_ERR_NONFINITE) set a sticky device error word; they are reported by
 * mpm_sync_errors() and by the calls documented as synchronising, after
 * which the context is poisoned: every later call returns that error until
 * the context is destroyed.  Outputs of a call whose work raised a device
 * error are unspecified.  A context is used by one host thread at a time.
 */
#ifndef MPM_H
#define MPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPM_OK 0
#define MPM_ERR_ARG (-1)       /* invalid argument (host-side check)        */
#define MPM_ERR_OOM (-2)       /* library scratch allocation failed          */
#define MPM_ERR_DOMAIN (-3)    /* a stencil base left [0, n-3] (or x not finite) */
#define MPM_ERR_INVERTED (-4)  /* det F <= 0                                 */
#define MPM_ERR_NONFINITE (-5) /* a non-finite value was produced            */
#define MPM_ERR_HIP (-6)       /* a HIP runtime call failed                  */
#define MPM_ERR_STATE (-7)     /* call out of order (e.g. no tape)           */

typedef struct mpm_ctx mpm_ctx;

/* One scene (HOST).  Physical meaning as in Table I: dt, E, nu, rho, V0 =
 * V_p^0 (equal for all particles), particle mass m_p = rho * V0.  Nodes
 * closer than `wall` to the box faces (index < wall or >= n - wall on any
 * axis) are wall nodes; after gravity their velocity is
 *   bc = 0: set to zero (sticky walls);
 *   bc = 1: passed through the friction projection of the supplement's
 *           friction projection gradients, (L), with coefficient `friction`
 *           (0 = frictionless slip): once per face whose band holds the
 *           node, in axis order, low face first, with the face's inward
 *           normal (+e_a at the low face, -e_a at the high face) and
 *           epsilon = 1e-12 under the tangential norm.
 * The reverse pass applies the reverse of (L) on those nodes. */
typedef struct mpm_scene {
  int32_t dim;         /* 2 or 3 (all scenes of a context alike)           */
  int32_t n_grid;      /* n: nodes per axis, dx = 1/n; n >= 3               */
  int32_t n_particles; /* N_s >= 0                                          */
  int32_t n_act;       /* actuators of this scene, 0..MPM_MAX_ACT           */
  int32_t wall;        /* wall thickness in nodes, >= 0                     */
  int32_t bc;          /* wall condition: 0 sticky, 1 friction projection   */
  float dt, E, nu, rho, V0;
  float gravity[3];    /* acceleration (only the first d entries are used)  */
  float act_axis[3];   /* sigma_pa = s_j diag(act_axis)                     */
  float friction;      /* coefficient c of (L), >= 0 (bc = 1)               */
} mpm_scene;

#define MPM_MAX_ACT 4096

/* Tuning options (HOST, nullable = defaults). */
typedef struct mpm_opts {
  int32_t tile;        /* cells per tile edge for binning; 0 = default
                          (8 in 2D, 4 in 3D)                                 */
  int32_t sort;        /* rollouts reorder particles by tile; 1 = yes
                          (default), 0 = keep the caller's order             */
  int32_t scatter;     /* binned scatters: 0 = default (3 when a tile has
                          64 cells, else 1); 1 = per-particle LDS atomics;
                          2 = per-cell register accumulation in bin order;
                          3 = per-cell accumulation after an in-LDS sort of
                          each tile by current cell (insensitive to drift)  */
  int32_t recompute_grids; /* checkpointed rollouts: 0 = keep every
                          substep's grid (m, p) on the tape so the reverse
                          pass recomputes states with G2P only (default);
                          1 = keep only states and recompute grids too      */
  int32_t graphs;      /* 1: rollouts replay hipGraphs of their inner loops
                          (captured once per tape layout on a library-owned
                          stream, launched on the context's stream); kernel
                          timing (mpm_profile) turns them off; 0 = eager     */
  int32_t fusion;      /* 3D binned rollouts: 0 = fuse each G2P with the next
                          substep's P2G (default); 1 = run every kernel
                          separately; 2 = also fuse each reverse gather with
                          the previous substep's adjoint scatter (two
                          workgroups per CU: slower on the measured scenes)  */
  int32_t deterministic; /* 1: binned rollouts are bitwise reproducible: the
                          binning ranks a cell's particles by index, the
                          scatters add a cell's records in a fixed order and
                          dL/ds is summed per actuator in a fixed order (needs
                          sort = 1 and the sorted scatter, i.e. the default
                          tile); particles that drift beyond their tile box's
                          one cell of slack still add with float atomics, so
                          a rollout is reproducible while none does; 0 = off */
  int32_t persistent;  /* 1: the binned rollouts' grid kernels run as
                          persistent workgroups (eight one-wave workgroups per
                          CU, each looping over its XCD's share of the node
                          tiles) instead of one workgroup per node tile    */
  int32_t rebin;       /* 1: sorted rollouts with uniform checkpoints
                          (1 <= ckpt_k < T) bin the particles again at every
                          checkpoint (the reverse pass uses each segment's
                          binning), so particles that travel stay within their
                          tile box's slack; 2: at the checkpoints where more
                          than 0.5% of the last segment's particle-substeps
                          scattered beyond their tile box's slack (global
                          atomics; the count is read back at every
                          checkpoint); re-binning waits for the device, so
                          such rollouts are never replayed as hipGraphs;
                          ignored with a material field or a controller
                          (binned once then); 0 = once per rollout          */
  int32_t reserved[1]; /* must be 0                                         */
} mpm_opts;

/* Particle state or its adjoint (DEVICE pointers, layout above). */
typedef struct mpm_state {
  float *x, *v, *C, *F;
} mpm_state;

/* Create a context for `n_scenes` scenes (HOST array).  `act_id` (HOST,
 * int32 [N_tot], nullable = all passive) gives each particle's actuator
 * within its scene, -1 for passive particles; it is copied.  `stream` is a
 * hipStream_t (NULL = the null stream) on which all work of the context is
 * queued.  Allocates the grids and scratch; synchronises the stream once.
 * Errors: MPM_ERR_ARG (bad scene or id), MPM_ERR_OOM, MPM_ERR_HIP. */
int mpm_init(mpm_ctx **out, const mpm_scene *scenes, int n_scenes,
             const int32_t *act_id, void *stream, const mpm_opts *opts);

/* Release every library allocation (after synchronising the stream). */
void mpm_destroy(mpm_ctx *ctx);

/* Change the stream of later work (hipStream_t, NULL = null stream). */
int mpm_set_stream(mpm_ctx *ctx, void *stream);

/* Sizes of the context: N_tot, n_act_tot, total grid nodes. Any may be NULL. */
int mpm_info(const mpm_ctx *ctx, int64_t *n_particles, int32_t *n_act,
             int64_t *n_nodes);

/* One substep (section III, steps 1-3; gravity and walls as in mpm_scene):
 *   P2G:  m_i = sum_p N m_p,  p_i = sum_p N [m_p v_p + G_p (x_i - x_p)],
 *         G_p = -(4/dx^2) dt V0 (P(F_p) + F_p sigma_pa) F_p^T + m_p C_p;
 *   grid: v_i = p_i/m_i + dt g (m_i > 0, else 0), 0 on wall nodes;
 *   G2P:  v' = sum_i N v_i,  C' = (4/dx^2) sum_i N v_i (x_i - x_p)^T,
 *         F' = (I + dt C') F,  x' = x + dt v'.
 * P(F) is the compressible neo-Hookean PK1 stress with Lame parameters from
 * (E, nu).  `act_n` is DEVICE [n_act_tot] (NULL when n_act_tot = 0).
 * `s_np1` may equal `s_n` (in place).  The grid of this step stays readable
 * through mpm_get_grid until the next call. */
int mpm_step_forward(mpm_ctx *ctx, const mpm_state *s_n, const float *act_n,
                     mpm_state *s_np1);

/* Allocation-free mpm_step_forward, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  One scene, one substep (the same P2G, grid operations
 * and G2P kernels as mpm_step_forward), no context: nothing is allocated,
 * freed or synchronised.  The grid, the scene's descriptors and a checked
 * copy of the actuator ids live in one static device region per GPU (about
 * 11 MB, held until the process ends) whose limits are
 * MPM_NOALLOC_MAX_PARTICLES particles and MPM_NOALLOC_MAX_NODES grid nodes;
 * larger scenes are rejected with MPM_ERR_ARG before any launch.
 *   scene   HOST descriptor, checked as by mpm_init (dim 2 or 3).
 *   act_id  DEVICE int32 [N] (nullable = all passive): each particle's
 *           actuator in [-1, n_act); an id outside that range is taken as
 *           passive and sets bit 8 of *err.
 *   s_n, s_np1, act_n  as for mpm_step_forward (DEVICE, ld = N; s_np1 may
 *           equal s_n; act_n nullable only when n_act = 0).
 *   err     DEVICE uint32, caller-owned: the kernels OR in 1 (a stencil base
 *           left the grid), 2 (det F <= 0), 4 (non-finite result), 8 (bad
 *           actuator id); the caller clears it and reads it after the stream.
 *   stream  hipStream_t on which the work is queued (asynchronous).
 * Every call on one GPU shares that GPU's region, which keeps the last
 * call's grid (the next call clears what must start at zero): calls that
 * overlap on one GPU (other streams, other host threads) race; calls queued
 * on one stream are ordered.  Returns MPM_ERR_ARG or MPM_ERR_HIP. */
#define MPM_NOALLOC_MAX_PARTICLES (1 << 20)
#define MPM_NOALLOC_MAX_NODES (1 << 18)
int mpm_step_forward_noalloc(const mpm_scene *scene, const int32_t *act_id,
                             const mpm_state *s_n, const float *act_n,
                             mpm_state *s_np1, uint32_t *err, void *stream);

/* Reverse of one substep (supplement (A)-(K)): given state n (`s_n`), its
 * actuation and the adjoint of state n+1 (`g_np1`), writes the adjoint of
 * state n to `g_n` (may equal `g_np1`) and ADDS dL/ds_j^n to `g_act_n`
 * (DEVICE [n_act_tot], nullable).  The forward grid of step n is recomputed
 * from `s_n`. */
int mpm_step_backward(mpm_ctx *ctx, const mpm_state *s_n, const float *act_n,
                      const mpm_state *g_np1, mpm_state *g_n, float *g_act_n);

/* T substeps from s0 with per-step actuation `act` (DEVICE [T][n_act_tot],
 * copied into the tape) writing the final state to sT.  The states needed by
 * the reverse pass are kept in a library-owned tape (the paper's "memo"):
 *   ckpt_k = 0  every state and grid is stored (no recompute);
 *   ckpt_k >= 1 every k-th state is stored and each segment of k substeps is
 *               recomputed from its checkpoint during the reverse pass (with
 *               the grids kept, on a second library stream, one segment
 *               ahead of the adjoint kernels);
 *   ckpt_k = -s (1 <= s <= MPM_MAX_REVOLVE_SLOTS) binomial checkpointing:
 *               s + 3 states and one grid whatever T (memory O(s N)); the
 *               reverse pass follows the schedule with the fewest recomputed
 *               substeps for s slots (mpm_revolve_steps), each substep's
 *               grid recomputed before its adjoint.
 * If `gT` is non-NULL the reverse pass runs at once and writes the adjoint
 * of s0 to `g0` and dL/ds [T][n_act_tot] to `g_act` (DEVICE, overwritten,
 * nullable); otherwise the tape is kept for mpm_rollout_backward.  The tape
 * lives until the next mpm_rollout or mpm_destroy.  Synchronises once
 * (after binning the particles) and returns device errors found up to then.
 * Errors: MPM_ERR_ARG, MPM_ERR_OOM, the device errors. */
int mpm_rollout(mpm_ctx *ctx, int T, int ckpt_k, const mpm_state *s0,
                const float *act, mpm_state *sT, const mpm_state *gT,
                mpm_state *g0, float *g_act);

#define MPM_MAX_REVOLVE_SLOTS 4096

/* Binomial checkpointing schedule (host-only, no context).  Reversing L
 * substeps from a held state with `slots` further state slots either
 * recomputes every state from the held one (slots = 0) or advances m
 * substeps, stores that state, reverses the last L - m with slots - 1 and
 * then the first m with `slots`.  mpm_revolve_steps returns the fewest
 * substeps this recomputes, F(L, c) = t L - C(c + 1 + t, t - 1) with
 * t = min{t : C(c + 1 + t, t) >= L} (Griewank's binomial count with c + 1
 * checkpoints); mpm_revolve_split the first split m attaining it (L >= 2,
 * slots >= 1).  -1 on invalid arguments. */
int64_t mpm_revolve_steps(int64_t L, int32_t slots);
int64_t mpm_revolve_split(int64_t L, int32_t slots);

/* Generation of the context's tape (HOST out): a counter bumped by every
 * mpm_rollout and mpm_rollout_ctrl (each replaces the tape, also when it
 * fails) and by mpm_set_materials (the reverse pass reads the material
 * field).  A caller that defers a reverse pass (an autograd graph) records
 * the value after its rollout and compares it before mpm_rollout_backward:
 * a different value means that reverse pass would differentiate another
 * rollout.  Errors: MPM_ERR_ARG (NULL argument). */
int mpm_tape_generation(const mpm_ctx *ctx, uint64_t *gen);

/* Binnings the forward pass of the current tape used (HOST out): 1 when the
 * particles were binned once (or the rollout is not binned), else 1 + the
 * checkpoints that sorted them into tiles again (mpm_opts.rebin; with
 * rebin = 2 the overflow count decides).  Errors: MPM_ERR_ARG (NULL
 * argument). */
int mpm_tape_binnings(const mpm_ctx *ctx, int32_t *n);

/* Reverse pass over the tape of the last mpm_rollout: chain rule across the
 * T substeps from dL/ds^T (`gT`) to dL/ds^0 (`g0`) and dL/ds [T][n_act_tot]
 * (`g_act`, overwritten, nullable).  MPM_ERR_STATE without a tape.  The tape
 * stays valid (the reverse pass may be run again with another gT). */
int mpm_rollout_backward(mpm_ctx *ctx, const mpm_state *gT, mpm_state *g0,
                         float *g_act);

/* Closed-loop controller (section IV, Control: a neural-network controller
 * fed with the positions and velocities of the robot's parts, here one dense
 * layer with tanh).  At every substep n of a rollout
 *   z^n = [target, for each component c: mean_{p in c} x_p^n,
 *                                        mean_{p in c} v_p^n]   (d (1 + 2 n_comp))
 *   a^n = tanh(W z^n + b)                                       ([n_act])
 * and a^n is the actuation s^n of that substep.  All pointers DEVICE:
 * comp_id int32 [N] (caller order; -1 = in no component; every component
 * needs at least one particle), W [n_act][d (1 + 2 n_comp)] row-major,
 * b [n_act], target [d].  Copied at the start of the rollout. */
typedef struct mpm_controller {
  int32_t n_comp;   /* 1 .. 48 / d */
  int32_t reserved;
  const int32_t *comp_id;
  const float *W, *b, *target;
} mpm_controller;

/* mpm_rollout with the actuation from the controller `ctl` instead of a
 * schedule.  One scene per context, 1 <= n_act <= 64.  `act` (DEVICE
 * [T][n_act], nullable) receives the actuation the controller produced.
 * With `gT` the reverse pass runs at once: `g0` = dL/dS^0 including the
 * controller's dependence on the state, `g_act` [T][n_act] = dL/ds^n
 * (partial, state held fixed), `g_W` [n_act][nz] and `g_b` [n_act] =
 * dL/dW, dL/db (all DEVICE, overwritten, the last three nullable).  The
 * G2P + P2G fusion of 3D rollouts is not used (a^{n+1} needs the means of
 * S^{n+1} first).  Synchronises to read the component ids.  Errors:
 * MPM_ERR_ARG (limits above, bad ids, empty component), MPM_ERR_OOM, the
 * device errors. */
int mpm_rollout_ctrl(mpm_ctx *ctx, int T, int ckpt_k, const mpm_state *s0,
                     const mpm_controller *ctl, mpm_state *sT, float *act,
                     const mpm_state *gT, mpm_state *g0, float *g_act,
                     float *g_W, float *g_b);

/* Reverse pass over the tape of the last mpm_rollout_ctrl (MPM_ERR_STATE if
 * the last rollout had no controller).  mpm_rollout_backward on such a tape
 * returns the same g0 and g_act without dL/dW, dL/db. */
int mpm_rollout_ctrl_backward(mpm_ctx *ctx, const mpm_state *gT, mpm_state *g0,
                              float *g_act, float *g_W, float *g_b);

/* Per-scene horizons (batched requests of different lengths): scene s is
 * held fixed from substep t_end[s] on, so a rollout of T >= t_end[s]
 * substeps returns its state after t_end[s] substeps, and the reverse pass
 * seeded at T returns the gradients of a loss on that state (the substeps
 * past the horizon are the identity and add nothing to dL/ds).  t_end: HOST
 * int32 [n_scenes], each >= 0; NULL removes every horizon.  Copied on the
 * context's stream; invalidates the tape.  Not combined with a closed-loop
 * controller (mpm_rollout_ctrl returns MPM_ERR_ARG). */
int mpm_set_horizons(mpm_ctx *ctx, const int32_t *t_end);

/* Per-particle materials (the co-design and system-identification uses of
 * section IV: a stiffness or density field instead of one material per
 * scene).  E_p, rho_p: DEVICE float [N_tot] in caller order, each nullable
 * (NULL = the scene's E or rho); both NULL switches the field off.  The
 * particle's Lame parameters follow from E_p and its scene's nu, its mass is
 * rho_p V0.  The values are copied by a kernel queued on the context's
 * stream (keep E_p, rho_p valid until the stream reaches it); they apply to
 * every later forward and reverse call (set them before a rollout and keep
 * them until its reverse pass).  With a field, the binned P2G's records carry each particle's
 * mass, the adjoint gather reads each particle's material, and 3D rollouts
 * do not fuse G2P with the next P2G. */
int mpm_set_materials(mpm_ctx *ctx, const float *E_p, const float *rho_p);

/* dL/dE_p and dL/drho_p (DEVICE float [N_tot], caller order, overwritten,
 * each nullable) accumulated by the last reverse pass (mpm_rollout with gT,
 * mpm_rollout_backward, mpm_rollout_ctrl(_backward) or mpm_step_backward):
 * summed over its substeps, through the stress (mu_p, la_p) and the mass
 * (m_i, m_p v_p and the m_p C_p part of G_p).  MPM_ERR_STATE without a
 * material field or before any reverse pass since it was set. */
int mpm_material_grad(mpm_ctx *ctx, float *g_E, float *g_rho);

/* Copy the grid of the last mpm_step_forward (DEVICE, caller-owned,
 * nullable): m [G], p [d][G], v [d][G] with G the total node count (scenes
 * concatenated in order, each n_s^d nodes).  Stream-ordered copy. */
int mpm_get_grid(mpm_ctx *ctx, float *m, float *p, float *v);

/* Sinusoid actuation bank (the actuation schedule of the paper's
 * controllers, open-loop form): act[n][j] = sum_k amp[j][k]
 * sin(2 pi freq[k] n dt + phase[j][k]), n < T, j < n_act, k < n_freq.
 * DEVICE arrays: freq [n_freq], amp/phase [n_act][n_freq], act [T][n_act].
 * `stream` is a hipStream_t.  Stateless (no context). */
int mpm_act_bank_forward(void *stream, int T, int n_act, int n_freq, float dt,
                         const float *freq, const float *amp,
                         const float *phase, float *act);

/* Its reverse: g_amp, g_phase [n_act][n_freq] (DEVICE, overwritten) from
 * g_act [T][n_act]. */
int mpm_act_bank_backward(void *stream, int T, int n_act, int n_freq,
                          float dt, const float *freq, const float *amp,
                          const float *phase, const float *g_act,
                          float *g_amp, float *g_phase);

/* Synchronise the context's stream and return the first device-side error
 * (MPM_OK if none).  A non-zero result poisons the context. */
int mpm_sync_errors(mpm_ctx *ctx);

/* Kernel timing with HIP events on the context's stream.  `mask` selects
 * the kernels to bracket (bit k = kernel id k below; 0 = off).  Each
 * selected launch records a start and a stop event; mpm_profile_read
 * synchronises the stream, returns per-kernel launch counts and summed
 * milliseconds (HOST arrays of MPM_NUM_KERNELS entries, nullable) and
 * resets the accumulators.  Events add a small gap per bracketed launch. */
#define MPM_K_P2G 0
#define MPM_K_GRID 1
#define MPM_K_G2P 2
#define MPM_K_ADJ_SCATTER 3
#define MPM_K_ADJ_GRID 4
#define MPM_K_ADJ_GATHER 5
#define MPM_K_G2P_P2G 6 /* G2P of substep n fused with P2G of n+1 (3D rollouts) */
#define MPM_K_ADJ_FUSED 7 /* reverse gather of substep n fused with the adjoint
                             scatter of n-1 (3D rollouts) */
#define MPM_NUM_KERNELS 8
int mpm_profile(mpm_ctx *ctx, uint32_t mask);
int mpm_profile_read(mpm_ctx *ctx, int64_t *count, double *ms);

/* Static description of an error code. */
const char *mpm_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* MPM_H */
