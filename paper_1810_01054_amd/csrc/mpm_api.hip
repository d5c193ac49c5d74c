// mpm_api.hip -- host implementation of the libmpm C ABI (include/mpm.h).
//
// One context = a fixed batch of scenes of one dimension.  All kernels of a
// substep cover every scene of the batch in one launch (chunks carry their
// scene).  Rollouts bin the particles once (tile / rank / cell order), run on
// library-owned sorted copies, keep a tape of checkpoints (or of every state
// and grid), and un-permute results on the way out.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/mpm.h"
#include "mpm_internal.h"

using namespace mpm;

namespace {

// controller limits: 2 d n_comp state entries (component means) at most
// CTL_MAX_ZS, at most CTL_MAX_ACT actuators
constexpr int CTL_MAX_ZS = 96;
constexpr int CTL_MAX_COMP = CTL_MAX_ZS / 4;
constexpr int CTL_MAX_ACT = 64;
constexpr int CTL_MAX_NZ = 3 + CTL_MAX_ZS;

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

// One binning of the particles (bin_particles): per-tile counts and ranges,
// the sorted order with its gather chunks, the non-empty tiles.  perm:
// sorted position -> caller index; act, pscene: actuator and scene of each
// sorted particle; rel (re-bins): sorted position -> position in the
// previous binning's order.
struct BinSet {
  int *tile_cnt = nullptr, *tile_start = nullptr, *perm = nullptr, *act = nullptr;
  int *tile_list = nullptr, *pscene = nullptr, *rel = nullptr;
  int *nt_cand = nullptr;  // 3D node tiles: covering tiles with particles [n_nt][8]
  Chunk *chunks = nullptr;
  int n_chunks = 0, n_ne = 0;
  bool owned = false;  // buffers allocated for this set (re-bins)
};

}  // namespace

struct mpm_ctx {
  int dim = 0;
  int n_scenes = 0;
  int64_t N = 0;        // total particles
  int n_act = 0;        // total actuators
  int64_t G = 0;        // total grid nodes
  int tile = 0;
  int sort = 1;
  int scatter_mode = 1;  // binned scatters: 1 atomics, 2 per-cell, 3 sorted per-cell
  int keep_grids = 1;    // checkpointed tapes keep every substep's grid
  int use_graphs = 0;    // rollouts replay captured hipGraphs
  int fuse_forward = 1;  // 3D binned rollouts: G2P fused with the next P2G
  int fuse_reverse = 0;  // 3D binned reverse: gather fused with the previous scatter
  int det = 0;           // deterministic sums (binned rollouts)
  bool horizons = false; // some scene has a horizon (mpm_set_horizons)
  int persistent = 0;    // persistent node-tile grid kernels
  int use_nt = 0;        // node-tile grid kernels (sorted scatter, 64-cell tiles)
  int n_nt = 0;          // node tiles of all scenes
  int *d_nt_scene = nullptr, *d_nt_dirty = nullptr;
  int *d_cell_start = nullptr, *d_cell_list = nullptr;  // det binning
  float *sb_part = nullptr;  // det: per-particle dL/ds of one substep
  int *d_act_scene = nullptr;  // det: scene of each actuator

  // captured inner loops of rollouts (forward, reverse)
  struct GraphKey {
    int T = 0, k = 0, memo = 0, grids_all = 0, sorted = 0, nch = 0, nne = 0, ctl = 0, rev = 0;
    int mat = 0;  // a per-particle material field selects other kernels
    const void *p[8] = {};
    bool operator==(const GraphKey &o) const {
      if (T != o.T || k != o.k || memo != o.memo || grids_all != o.grids_all ||
          sorted != o.sorted || nch != o.nch || nne != o.nne || ctl != o.ctl ||
          rev != o.rev || mat != o.mat)
        return false;
      for (int i = 0; i < 8; ++i)
        if (p[i] != o.p[i]) return false;
      return true;
    }
  };
  struct GraphSlot {
    hipGraphExec_t exec = nullptr;
    GraphKey key;
    bool valid = false;
  } gfwd, gbwd;
  hipStream_t cap_stream = nullptr;
  // second library stream for the reverse pass's recompute, which runs one
  // segment ahead of the adjoint kernels (default priority)
  hipStream_t aux_stream = nullptr;
  hipEvent_t ev_start = nullptr, ev_recomp = nullptr, ev_adj = nullptr;
  hipStream_t stream = nullptr;
  int poisoned = 0;
  // bumped by every call that replaces the tape or the material field the
  // reverse pass reads (mpm_tape_generation)
  uint64_t tape_gen = 0;

  std::vector<DevScene> h_scenes;
  DevScene *d_scenes = nullptr;
  std::vector<int> h_act_id;

  // caller-order chunks (step calls, unsorted rollouts)
  Chunk *d_chunks_user = nullptr;
  int n_chunks_user = 0;
  GridBlock *d_gblocks = nullptr;
  int n_gblocks = 0;
  int *d_act_id = nullptr;   // caller order
  int *d_pscene = nullptr;   // scene of each particle (caller order)

  // grids
  float *gm = nullptr, *gp = nullptr, *gv = nullptr;
  float *vbar = nullptr, *pbar = nullptr, *mbar = nullptr;
  double *gact = nullptr;    // [gact_cap] FP64 accumulators for dL/ds
  int64_t gact_cap = 0;
  unsigned *d_err = nullptr;

  // step_backward scratch: one state (for C^{n+1})
  float *scratch = nullptr;

  // binning
  int n_tiles = 0;
  int *d_tile_scene = nullptr, *d_tile_cnt = nullptr, *d_cell_cnt = nullptr;
  int *d_ptile = nullptr, *d_pcell = nullptr, *d_prank = nullptr;
  int *d_tile_start = nullptr, *d_nch = nullptr, *d_chunk_start = nullptr;
  int *d_perm = nullptr, *d_act_sorted = nullptr;
  Chunk *d_chunks_sorted = nullptr;
  int n_chunks_sorted = 0;
  float *d_part = nullptr;   // tile boxes [n_tiles][d+1][S^d]
  int *d_tile_flag = nullptr, *d_tile_pos = nullptr, *d_tile_list = nullptr;
  int n_tiles_ne = 0;        // non-empty tiles (binned rollouts)
  // binnings: [0] aliases the buffers above; with re-binning, [j] is the
  // binning of checkpoint segment j of the current tape
  std::vector<BinSet> bins;
  int cur_bin = 0;
  int rebin = 0;             // 1: re-bin at every checkpoint, 2: when particles overflow
  int n_bins = 1;            // binnings of the current tape
  int *d_over = nullptr;     // particles scattered beyond their tile box's slack
  int *h_over = nullptr;     // (pinned host copy, read at checkpoints)

  // tape
  struct Tape {
    int valid = 0, T = 0, k = 0, memo = 0, sorted = 0, grids_all = 0;
    int rev = 0;              // > 0: binomial checkpointing with rev slots
    int rev_spine = 0;        // its first-descent checkpoints are intact
    int rebin = 0;            // re-binned tape: segment j uses bins[seg_bin[j]]
    std::vector<int> seg_bin; // binning of each checkpoint segment
    float *states = nullptr;  // slots of one state each
    int64_t state_cap = 0;    // slots allocated
    float *grids = nullptr;   // slots of (1 + d) * G floats (m, p)
    int64_t grid_cap = 0;
    float *act = nullptr;     // [T][n_act]
    int64_t act_cap = 0;
    float *pp = nullptr;      // two ping-pong states
    float *adj = nullptr;     // two adjoint states
  } tape;

  // per-particle materials: (mu, la, m_p) [3][N] in caller and tape order,
  // and the reverse pass's dL/dmu, dL/dla, dL/dm_p [3][N]
  float *mat_user = nullptr, *mat_sorted = nullptr, *gmat = nullptr;
  int has_mat = 0, gmat_sorted = 0, gmat_valid = 0;

  // closed-loop controller of the current tape (one scene; section IV)
  struct Ctl {
    int on = 0, n_comp = 0, nz = 0;
    int *comp = nullptr;       // component of each particle (tape order) [N]
    float *inv_cnt = nullptr;  // [CTL_MAX_COMP]
    float *W = nullptr, *b = nullptr, *target = nullptr;  // copies
    float *partial = nullptr;  // [2 d n_comp][partial_rows] (entry-major)
    int partial_rows = 0;
    double *sums = nullptr;    // [CTL_MAX_ZS]
    unsigned *done = nullptr;  // reduction counter (zero between launches)
    double *gW = nullptr, *gb = nullptr;  // FP64 accumulators
    float *Z = nullptr;        // tape of z^n [T][nz]
    int64_t Z_cap = 0;
  } ctl;

  // kernel timing (mpm_profile)
  struct Prof {
    uint32_t mask = 0;
    std::vector<hipEvent_t> pool;  // start/stop pairs
    size_t used = 0;
    std::vector<int> kid;          // kernel id of each pair
    int64_t count[MPM_NUM_KERNELS] = {};
    double ms[MPM_NUM_KERNELS] = {};
  } prof;

  int64_t state_floats() const {
    return (int64_t)(2 * dim + 2 * dim * dim) * N;
  }
};

namespace {

int hip_ok(hipError_t e) { return e == hipSuccess ? MPM_OK : MPM_ERR_HIP; }

// Host-side checks of one scene descriptor (mpm_init and the
// allocation-free step).
bool scene_valid(const mpm_scene &S, int dim) {
  if (S.dim != dim || S.n_grid < 3 || S.n_particles < 0 || S.n_act < 0 ||
      S.n_act > MPM_MAX_ACT || S.wall < 0 || (S.bc != 0 && S.bc != 1))
    return false;
  if (S.bc == 1 && !(S.friction >= 0.0f && std::isfinite(S.friction))) return false;
  if (!(S.dt > 0.0f) || !(S.V0 > 0.0f) || !(S.rho > 0.0f) || !(S.E >= 0.0f) ||
      !(S.nu > -1.0f && S.nu < 0.5f) || !std::isfinite(S.dt) || !std::isfinite(S.E))
    return false;
  return true;
}

// The kernels' copy of a scene: derived constants (dx = 1/n, D = 4/dx^2,
// Lame parameters, m_p = rho V0, the stress factor of G_p); offsets zero.
DevScene dev_scene(const mpm_scene &S, int tile) {
  DevScene d{};
  d.n = S.n_grid;
  d.np = S.n_particles;
  d.n_act = S.n_act;
  d.wall = S.wall;
  d.bc = S.bc;
  d.nu = S.nu;
  d.fric = S.bc == 1 ? S.friction : 0.0f;
  d.nt = (int)((S.n_grid - 2 + tile - 1) / tile);
  d.nnt = S.n_grid / tile + 1;
  d.t_end = INT32_MAX;
  d.dt = S.dt;
  d.dx = 1.0f / (float)S.n_grid;
  d.inv_dx = (float)S.n_grid;
  d.Dinv = 4.0f * (float)S.n_grid * (float)S.n_grid;
  d.mu = S.E / (2.0f * (1.0f + S.nu));
  d.la = S.E * S.nu / ((1.0f + S.nu) * (1.0f - 2.0f * S.nu));
  d.mp = S.rho * S.V0;
  d.V0 = S.V0;
  d.kG = -d.Dinv * S.dt * S.V0;
  for (int a = 0; a < 3; ++a) {
    d.g[a] = S.gravity[a];
    d.axis[a] = S.act_axis[a];
  }
  return d;
}

template <typename T>
int dmalloc(T **p, int64_t count, hipStream_t st) {
  // stream-ordered allocation: no device-wide synchronisation, so contexts
  // can come and go while other contexts' work runs on other streams
  *p = nullptr;
  if (count <= 0) count = 1;
  hipError_t e = hipMallocAsync((void **)p, sizeof(T) * (size_t)count, st);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return MPM_ERR_OOM;
  }
  return MPM_OK;
}

template <typename T>
void dfree(T *&p, hipStream_t st) {
  if (p) (void)hipFreeAsync((void *)p, st);
  p = nullptr;
}

#define RC(x)                  \
  do {                         \
    int _rc = (x);             \
    if (_rc) return _rc;       \
  } while (0)

State state_at(const mpm_ctx *c, float *base) {
  const int64_t N = c->N, d = c->dim;
  State s;
  s.x = base;
  s.v = base + d * N;
  s.C = base + 2 * d * N;
  s.F = base + 2 * d * N + d * d * N;
  return s;
}

CState cs(const State &s) { return CState{s.x, s.v, s.C, s.F}; }
CState cs(const mpm_state &s) { return CState{s.x, s.v, s.C, s.F}; }
State st(const mpm_state &s) { return State{s.x, s.v, s.C, s.F}; }

bool state_ok(const mpm_ctx *c, const mpm_state *s) {
  if (!s) return false;
  if (c->N == 0) return true;
  return s->x && s->v && s->C && s->F;
}

int check_ctx(mpm_ctx *c) {
  if (!c) return MPM_ERR_ARG;
  if (c->poisoned) return c->poisoned;
  return MPM_OK;
}

// ---- kernel timing ---------------------------------------------------------

constexpr size_t PROF_MAX_EVENTS = 1 << 20;

hipEvent_t prof_event(mpm_ctx *c) {
  auto &P = c->prof;
  if (P.used == P.pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    P.pool.push_back(e);
  }
  return P.pool[P.used++];
}

// Bracket one launch of kernel k with events (when selected by the mask).
struct ProfScope {
  mpm_ctx *c;
  int k;
  bool on;
  ProfScope(mpm_ctx *c_, int k_) : c(c_), k(k_) {
    on = (c->prof.mask >> k & 1u) && c->prof.used + 2 <= PROF_MAX_EVENTS;
    if (on) {
      hipEvent_t e = prof_event(c);
      on = e && hipEventRecord(e, c->stream) == hipSuccess;
    }
  }
  ~ProfScope() {
    if (!on) return;
    hipEvent_t e = prof_event(c);
    if (e && hipEventRecord(e, c->stream) == hipSuccess) c->prof.kid.push_back(k);
    else c->prof.used -= e ? 2 : 1;
  }
};

int decode_err(unsigned bits) {
  if (bits & EB_DOMAIN) return MPM_ERR_DOMAIN;
  if (bits & EB_INVERTED) return MPM_ERR_INVERTED;
  if (bits & EB_NONFINITE) return MPM_ERR_NONFINITE;
  return MPM_OK;
}

int read_err(mpm_ctx *c) {
  unsigned bits = 0;
  RC(hip_ok(hipMemcpyAsync(&bits, c->d_err, sizeof(unsigned),
                           hipMemcpyDeviceToHost, c->stream)));
  RC(hip_ok(hipStreamSynchronize(c->stream)));
  int e = decode_err(bits);
  if (e) c->poisoned = e;
  return e;
}

// ---- the three kernels of one forward substep ------------------------------

BinSet &bin(mpm_ctx *c) { return c->bins[(size_t)c->cur_bin]; }

TileInfo tile_info(mpm_ctx *c) {
  const BinSet &b = bin(c);
  TileInfo t;
  t.cnt = b.tile_cnt;
  t.start = b.tile_start;
  t.scene = c->d_tile_scene;
  t.part = c->d_part;
  t.B = c->tile;
  t.list = b.tile_list;
  t.nt_dirty = c->use_nt ? c->d_nt_dirty : nullptr;
  t.n_over = c->tape.rebin == 2 ? c->d_over : nullptr;
  return t;
}

// `tiles`: particles are binned (rollouts); scatters go through tile boxes.
int fwd_p2g(mpm_ctx *c, bool tiles, const Chunk *chunks, int n_chunks,
            CState s, const int *act_id, const float *act, float *gm,
            float *gp, int n = 0) {
  P2GArgs a;
  a.n = n;
  a.scenes = c->d_scenes;
  a.chunks = chunks;
  a.n_chunks = n_chunks;
  a.s = s;
  a.ld = (int)c->N;
  a.act_id = act_id;
  a.act = act;
  a.gm = gm;
  a.gp = gp;
  a.G = c->G;
  a.err = c->d_err;
  a.tiles = tile_info(c);
  // per-particle materials: the sorted scatter's records then carry each
  // particle's mass (the per-cell mode falls back to per-tile LDS atomics)
  a.mat = c->has_mat ? (tiles ? c->mat_sorted : c->mat_user) : nullptr;
  a.det = tiles && c->det;
  ProfScope ps(c, MPM_K_P2G);
  if (tiles && c->scatter_mode == 3)
    return launch_p2g_sorted(c->dim, a, bin(c).n_ne, c->stream);
  a.tiles.list = nullptr;  // the other binned modes launch one block per tile
  if (tiles && c->scatter_mode == 2 && !c->has_mat)
    return launch_p2g_cell(c->dim, a, c->d_cell_cnt, c->n_tiles, c->stream);
  if (tiles) return launch_p2g_tile(c->dim, a, c->n_tiles, c->stream);
  return launch_p2g(c->dim, a, c->stream);
}

int fwd_grid(mpm_ctx *c, bool tiles, float *gm, float *gp, float *gv,
             int zero_mp, float *out_m = nullptr, float *out_p = nullptr) {
  GridArgs a;
  a.scenes = c->d_scenes;
  a.blocks = c->d_gblocks;
  a.n_blocks = c->n_gblocks;
  a.gm = gm;
  a.gp = gp;
  a.gv = gv;
  a.G = c->G;
  a.zero_mp = zero_mp;
  a.tile_cnt = tiles ? bin(c).tile_cnt : nullptr;
  a.part = tiles ? c->d_part : nullptr;
  a.B = c->tile;
  a.out_m = out_m;
  a.out_p = out_p;
  ProfScope ps(c, MPM_K_GRID);
  if (tiles && c->use_nt) {
    a.nt_scene = c->d_nt_scene;
    a.nt_dirty = c->d_nt_dirty;
    a.n_nt = c->n_nt;
    a.persist = c->persistent;
    a.nt_cand = bin(c).nt_cand;
    return launch_grid_nt(c->dim, a, c->stream);
  }
  return launch_grid(c->dim, a, c->stream);
}

int fwd_g2p(mpm_ctx *c, const Chunk *chunks, int n_chunks, CState s,
            State out, const float *gv, const float *gm = nullptr,
            const float *gp = nullptr, hipStream_t st = nullptr,
            bool ctl_sums = false, int n = 0) {
  G2PArgs a;
  a.n = n;
  a.scenes = c->d_scenes;
  a.chunks = chunks;
  a.n_chunks = n_chunks;
  a.s = s;
  a.out = out;
  a.ld = (int)c->N;
  a.gv = gv;
  a.gm = gm;
  a.gp = gp;
  a.G = c->G;
  a.err = c->d_err;
  if (ctl_sums) {  // the next substep's controller reads these rows
    if (c->ctl.partial_rows < n_chunks) return MPM_ERR_ARG;
    a.ctl_comp = c->ctl.comp;
    a.ctl_partial = c->ctl.partial;
    a.ctl_nzs = 2 * c->dim * c->ctl.n_comp;
    a.ctl_rows = n_chunks;  // rows = chunks, entry stride n_chunks
  }
  ProfScope ps(c, MPM_K_G2P);
  return launch_g2p(c->dim, a, st ? st : c->stream);
}

// G2P of substep n (state s, grid velocity gv) fused with the binned P2G of
// substep n+1 (actuation act1) into the tile boxes; writes state n+1.
int fwd_g2p_p2g(mpm_ctx *c, CState s, State out, const float *gv,
                const int *act_id, const float *act1, bool write_vc, int n) {
  G2P2GArgs a;
  a.n = n;
  a.write_vc = write_vc ? 1 : 0;
  a.scenes = c->d_scenes;
  a.s = s;
  a.out = out;
  a.ld = (int)c->N;
  a.gv = gv;
  a.act_id = act_id;
  a.act = act1;
  a.gm = c->gm;
  a.gp = c->gp;
  a.G = c->G;
  a.err = c->d_err;
  a.tiles = tile_info(c);
  a.mat = c->has_mat ? c->mat_sorted : nullptr;  // (binned rollouts only)
  a.det = c->det;
  ProfScope ps(c, MPM_K_G2P_P2G);
  return launch_g2p_p2g_sorted(c->dim, a, bin(c).n_ne, c->stream);
}

// ---- the kernels of one reverse substep ------------------------------------
// gm/gp: forward grid of step n (m, p).

// (A)-(C): adjoint of G2P, scattered into the tile boxes / vbar.
int bwd_scatter(mpm_ctx *c, bool tiles, const Chunk *chunks, int n_chunks,
                CState s, CState g1, int n = 0) {
  AdjScatterArgs r1;
  r1.n = n;
  r1.scenes = c->d_scenes;
  r1.chunks = chunks;
  r1.n_chunks = n_chunks;
  r1.s = s;
  r1.g1 = g1;
  r1.ld = (int)c->N;
  r1.vbar = c->vbar;
  r1.G = c->G;
  r1.err = c->d_err;
  r1.tiles = tile_info(c);
  r1.det = tiles && c->det;
  ProfScope ps(c, MPM_K_ADJ_SCATTER);
  if (tiles && c->scatter_mode == 3)
    return launch_adj_scatter_sorted(c->dim, r1, bin(c).n_ne, c->stream);
  r1.tiles.list = nullptr;
  if (tiles && c->scatter_mode == 2)
    return launch_adj_scatter_cell(c->dim, r1, c->d_cell_cnt, c->n_tiles, c->stream);
  if (tiles) return launch_adj_scatter_tile(c->dim, r1, c->n_tiles, c->stream);
  return launch_adj_scatter(c->dim, r1, c->stream);
}

// (D)-(E): adjoint of the grid operations (sums the tile boxes).
int bwd_grid(mpm_ctx *c, bool tiles, const float *gm, const float *gp) {
  AdjGridArgs r2;
  r2.scenes = c->d_scenes;
  r2.blocks = c->d_gblocks;
  r2.n_blocks = c->n_gblocks;
  r2.gm = gm;
  r2.gp = gp;
  r2.vbar = c->vbar;
  r2.pbar = c->pbar;
  r2.mbar = c->mbar;
  r2.gv = c->gv;
  r2.G = c->G;
  r2.tile_cnt = tiles ? bin(c).tile_cnt : nullptr;
  r2.part = tiles ? c->d_part : nullptr;
  r2.B = c->tile;
  ProfScope ps(c, MPM_K_ADJ_GRID);
  if (tiles && c->use_nt) {
    r2.nt_scene = c->d_nt_scene;
    r2.nt_dirty = c->d_nt_dirty;
    r2.n_nt = c->n_nt;
    r2.persist = c->persistent;
    r2.nt_cand = bin(c).nt_cand;
    return launch_adj_grid_nt(c->dim, r2, c->stream);
  }
  return launch_adj_grid(c->dim, r2, c->stream);
}

// (F)-(K): adjoint of P2G and of the particle update, gathered.
int bwd_gather(mpm_ctx *c, bool tiles, const Chunk *chunks, int n_chunks,
               CState s, const int *act_id, const float *act, CState g1,
               State g0, double *gact, int n = 0) {
  AdjGatherArgs r3;
  r3.n = n;
  r3.scenes = c->d_scenes;
  r3.chunks = chunks;
  r3.n_chunks = n_chunks;
  r3.s = s;
  r3.g1 = g1;
  r3.g0 = g0;
  r3.ld = (int)c->N;
  r3.act_id = act_id;
  r3.act = act;
  r3.pbar = c->pbar;
  r3.mbar = c->mbar;
  r3.gv = c->gv;
  r3.G = c->G;
  r3.gact = gact;
  r3.err = c->d_err;
  r3.mat = c->has_mat ? (tiles ? c->mat_sorted : c->mat_user) : nullptr;
  r3.gmat = c->has_mat ? c->gmat : nullptr;
  // deterministic mode: per-particle dL/ds, then a fixed-order sum
  const bool det_s = tiles && c->det && gact != nullptr && c->n_act > 0;
  if (det_s) {
    r3.gact = nullptr;
    r3.sb_part = c->sb_part;
  }
  {
    ProfScope ps(c, MPM_K_ADJ_GATHER);
    RC(launch_adj_gather(c->dim, r3, c->stream));
  }
  if (det_s)
    RC(launch_sbar_reduce(c->d_scenes, c->d_act_scene, c->n_act, bin(c).tile_start,
                          act_id, c->sb_part, c->dim, gact, c->stream));
  return MPM_OK;
}

int bwd_step(mpm_ctx *c, bool tiles, const Chunk *chunks, int n_chunks,
             CState s, const int *act_id, const float *act,
             const float *gm, const float *gp, CState g1, State g0,
             double *gact, int n = 0) {
  RC(bwd_scatter(c, tiles, chunks, n_chunks, s, g1, n));
  RC(bwd_grid(c, tiles, gm, gp));
  return bwd_gather(c, tiles, chunks, n_chunks, s, act_id, act, g1, g0, gact, n);
}

// The gather of reverse substep n fused with the scatter of substep n-1
// (3D binned rollouts): reads state n, the adjoint of state n+1 and x, F of
// state n-1; writes the adjoint of state n (g0, not aliasing g1).
int bwd_gather_scatter(mpm_ctx *c, CState s, CState sp, const int *act_id,
                       const float *act, CState g1, State g0, double *gact, int n) {
  AdjFusedArgs a;
  a.n = n;
  a.scenes = c->d_scenes;
  a.s = s;
  a.g1 = g1;
  a.g0 = g0;
  a.sp = sp;
  a.ld = (int)c->N;
  a.act_id = act_id;
  a.act = act;
  a.pbar = c->pbar;
  a.mbar = c->mbar;
  a.gv = c->gv;
  a.G = c->G;
  a.gact = gact;
  a.vbar = c->vbar;
  a.err = c->d_err;
  a.tiles = tile_info(c);
  a.det = c->det;
  const bool det_s = c->det && gact != nullptr && c->n_act > 0;
  if (det_s) {
    a.gact = nullptr;
    a.sb_part = c->sb_part;
  }
  {
    ProfScope ps(c, MPM_K_ADJ_FUSED);
    RC(launch_adj_gather_scatter(c->dim, a, bin(c).n_ne, c->stream));
  }
  if (det_s)
    RC(launch_sbar_reduce(c->d_scenes, c->d_act_scene, c->n_act, bin(c).tile_start,
                          act_id, c->sb_part, c->dim, gact, c->stream));
  return MPM_OK;
}

int ensure_gact(mpm_ctx *c, int64_t n) {
  if (n <= c->gact_cap) return MPM_OK;
  dfree(c->gact, c->stream);
  c->gact_cap = 0;
  RC(dmalloc(&c->gact, n, c->stream));
  c->gact_cap = n;
  return MPM_OK;
}

// ---- binning: sorted order, chunks per tile --------------------------------

// Bins the particles whose positions are `x` into `dst`.  prev == nullptr:
// x in the caller's order (the first binning of a tape: the node-tile flags
// are cleared); otherwise x is in prev's sorted order and dst.rel maps the
// new order to it.
int bin_particles(mpm_ctx *c, const float *x, BinSet &dst, const BinSet *prev = nullptr) {
  const int cpt = c->dim == 2 ? c->tile * c->tile : c->tile * c->tile * c->tile;
  hipStream_t s = c->stream;
  const int N = (int)c->N;
  RC(launch_fill_i32(c->d_cell_cnt, (int64_t)c->n_tiles * cpt, s));
  RC(launch_fill_i32(dst.tile_cnt, c->n_tiles, s));
  // node tiles flagged by particles beyond their box's slack, for this tape
  if (c->use_nt && !prev) RC(launch_fill_i32(c->d_nt_dirty, c->n_nt, s));
  SortArgs a;
  a.scenes = c->d_scenes;
  a.pscene = prev ? prev->pscene : c->d_pscene;
  a.N = N;
  a.x = x;
  a.ld = N;
  a.tile = c->tile;
  a.cell_cnt = c->d_cell_cnt;
  a.tile_cnt = dst.tile_cnt;
  a.ptile = c->d_ptile;
  a.pcell = c->d_pcell;
  a.prank = c->d_prank;
  a.err = c->d_err;
  RC(launch_sort_count(c->dim, a, s));
  // an invalid particle gets no slot in the permutation: stop here (before
  // any kernel reads the permutation) when counting found one
  RC(read_err(c));  // synchronises
  if (c->det) {
    // ranks in a cell by particle index instead of atomic arrival
    const int64_t ncell = (int64_t)c->n_tiles * cpt;
    RC(launch_scan_i32(c->d_cell_cnt, c->d_cell_start, (int)ncell, s));
    RC(launch_cell_fill(c->d_ptile, c->d_pcell, c->d_prank, c->d_cell_start, cpt, N,
                        c->d_cell_list, s));
    RC(launch_cell_sort(c->d_cell_start, (int)ncell, c->d_cell_list, c->d_prank, s));
  }
  RC(launch_scan_i32(dst.tile_cnt, dst.tile_start, c->n_tiles, s));
  if (dst.nt_cand)
    RC(launch_nt_cand(c->d_scenes, c->d_nt_scene, c->n_nt, dst.tile_cnt, dst.nt_cand, s));
  if (prev) {
    RC(launch_sort_place(c->dim, a, dst.tile_start, dst.rel, s));
    RC(launch_permute_i32(prev->perm, dst.perm, dst.rel, N, s));
  } else {
    RC(launch_sort_place(c->dim, a, dst.tile_start, dst.perm, s));
  }
  RC(launch_chunk_count(dst.tile_cnt, c->n_tiles, c->d_nch, s));
  RC(launch_scan_i32(c->d_nch, c->d_chunk_start, c->n_tiles, s));
  RC(launch_build_chunks(dst.tile_cnt, dst.tile_start, c->d_chunk_start,
                         c->d_tile_scene, c->n_tiles, dst.chunks, s));
  RC(launch_permute_i32(c->d_act_id, dst.act, dst.perm, N, s));
  if (dst.pscene) RC(launch_permute_i32(c->d_pscene, dst.pscene, dst.perm, N, s));
  if (c->has_mat)
    RC(launch_permute_rows(c->mat_user, c->mat_sorted, dst.perm, N, N, 3, 0, s));
  RC(launch_nonempty_flag(dst.tile_cnt, c->n_tiles, c->d_tile_flag, s));
  RC(launch_scan_i32(c->d_tile_flag, c->d_tile_pos, c->n_tiles, s));
  RC(launch_compact(c->d_tile_flag, c->d_tile_pos, c->n_tiles, dst.tile_list, s));
  int nch = 0, nne = 0;
  RC(hip_ok(hipMemcpyAsync(&nch, c->d_chunk_start + c->n_tiles, sizeof(int),
                           hipMemcpyDeviceToHost, s)));
  RC(hip_ok(hipMemcpyAsync(&nne, c->d_tile_pos + c->n_tiles, sizeof(int),
                           hipMemcpyDeviceToHost, s)));
  RC(read_err(c));  // synchronises
  dst.n_chunks = nch;
  dst.n_ne = nne;
  // launch the fullest tiles first: one workgroup per tile takes time
  // roughly in proportion to its particles, and the small tiles then fill
  // the last round of workgroup slots instead of trailing it
  if (nne > 1) {
    std::vector<int> cnt(c->n_tiles), list(nne);
    RC(hip_ok(hipMemcpyAsync(cnt.data(), dst.tile_cnt, sizeof(int) * c->n_tiles,
                             hipMemcpyDeviceToHost, s)));
    RC(hip_ok(hipMemcpyAsync(list.data(), dst.tile_list, sizeof(int) * nne,
                             hipMemcpyDeviceToHost, s)));
    RC(hip_ok(hipStreamSynchronize(s)));
    std::stable_sort(list.begin(), list.end(),
                     [&](int a, int b) { return cnt[a] > cnt[b]; });
    RC(hip_ok(hipMemcpyAsync(dst.tile_list, list.data(), sizeof(int) * nne,
                             hipMemcpyHostToDevice, s)));
    RC(hip_ok(hipStreamSynchronize(s)));  // `list` is host memory
  }
  return MPM_OK;
}

int permute_state_by(mpm_ctx *c, const mpm_state &src, State dst, const int *perm,
                     int scatter) {
  // gather: dst[i] = src[perm[i]];  scatter: dst[perm[i]] = src[i]
  const int d = c->dim, N = (int)c->N;
  RC(launch_permute_rows(src.x, dst.x, perm, N, N, d, scatter, c->stream));
  RC(launch_permute_rows(src.v, dst.v, perm, N, N, d, scatter, c->stream));
  RC(launch_permute_rows(src.C, dst.C, perm, N, N, d * d, scatter, c->stream));
  RC(launch_permute_rows(src.F, dst.F, perm, N, N, d * d, scatter, c->stream));
  return MPM_OK;
}

// between the caller's order and the current binning's
int permute_state(mpm_ctx *c, const mpm_state &src, State dst, int scatter) {
  return permute_state_by(c, src, dst, bin(c).perm, scatter);
}

int copy_state(mpm_ctx *c, const mpm_state &src, State dst) {
  const size_t vb = sizeof(float) * c->dim * c->N;
  const size_t mb = sizeof(float) * c->dim * c->dim * c->N;
  RC(hip_ok(hipMemcpyAsync(dst.x, src.x, vb, hipMemcpyDeviceToDevice, c->stream)));
  RC(hip_ok(hipMemcpyAsync(dst.v, src.v, vb, hipMemcpyDeviceToDevice, c->stream)));
  RC(hip_ok(hipMemcpyAsync(dst.C, src.C, mb, hipMemcpyDeviceToDevice, c->stream)));
  RC(hip_ok(hipMemcpyAsync(dst.F, src.F, mb, hipMemcpyDeviceToDevice, c->stream)));
  return MPM_OK;
}

mpm_state ms(const State &s) { return mpm_state{s.x, s.v, s.C, s.F}; }

// ---- tape ------------------------------------------------------------------

int ensure_tape(mpm_ctx *c, int64_t states, int64_t grids, int64_t act) {
  auto &t = c->tape;
  const int64_t sf = c->state_floats();
  const int64_t gf = (int64_t)(1 + c->dim) * c->G;
  if (states > t.state_cap) {
    dfree(t.states, c->stream);
    t.state_cap = 0;
    RC(dmalloc(&t.states, states * sf, c->stream));
    t.state_cap = states;
  }
  if (grids > t.grid_cap) {
    dfree(t.grids, c->stream);
    t.grid_cap = 0;
    RC(dmalloc(&t.grids, grids * gf, c->stream));
    // grid kernels skip nodes no particle reached; those keep these zeros
    RC(launch_fill_f32(t.grids, grids * gf, c->stream));
    t.grid_cap = grids;
  }
  if (act > t.act_cap) {
    dfree(t.act, c->stream);
    t.act_cap = 0;
    RC(dmalloc(&t.act, act, c->stream));
    t.act_cap = act;
  }
  if (!t.pp) RC(dmalloc(&t.pp, 2 * sf, c->stream));
  if (!t.adj) RC(dmalloc(&t.adj, 2 * sf, c->stream));
  return MPM_OK;
}

// Slot layout:
//   memo:  states[n] = S^n (n = 0..T), grids[n] = grid of step n (n < T)
//   ckpt:  states[j] = S^{min(j k, T)} (j = 0..ceil(T/k)), then k segment
//          slots; grids[0..k) = grids of the segment being reversed.
struct Layout {
  int T, k, memo, ncp;
};

float *slot_state(mpm_ctx *c, int64_t i) {
  return c->tape.states + i * c->state_floats();
}
float *slot_grid(mpm_ctx *c, int64_t i) {
  return c->tape.grids + i * (int64_t)(1 + c->dim) * c->G;
}

const Chunk *cur_chunks(mpm_ctx *c, int *n) {
  if (c->tape.sorted) {
    *n = bin(c).n_chunks;
    return bin(c).chunks;
  }
  *n = c->n_chunks_user;
  return c->d_chunks_user;
}

const int *cur_act_id(mpm_ctx *c) {
  return c->tape.sorted ? bin(c).act : c->d_act_id;
}

// forward state S^n for the rollout (ckpt mode; n is a checkpoint or lives in
// the ping-pong pair)
// First substep of the last segment of a checkpointed tape.
int last_seg_start(const Layout &L) { return L.T > 0 ? ((L.T - 1) / L.k) * L.k : 0; }

// Checkpointed tapes with stored grids keep the states of their last
// segment from the forward pass (its own bank, 2): the reverse pass starts
// on it at once instead of first recomputing it.
bool keeps_last_segment(const mpm_ctx *c, const Layout &L, int n) {
  return c->tape.grids_all && !L.memo && !c->tape.rev && n > last_seg_start(L) && n < L.T;
}

float *fwd_slot(mpm_ctx *c, const Layout &L, int n) {
  if (c->tape.rev) return slot_state(c, n == L.T && n > 0 ? c->tape.rev + 2 : 0);
  if (L.memo) return slot_state(c, n);
  if (n % L.k == 0) return slot_state(c, n / L.k);
  if (n == L.T) return slot_state(c, L.ncp - 1);
  if (keeps_last_segment(c, L, n))
    return slot_state(c, L.ncp + 2 * (int64_t)L.k + (n - last_seg_start(L)));
  return c->tape.pp + (int64_t)(n & 1) * c->state_floats();
}

// Run `body` (stream-ordered launches on c->stream only) directly, or as a
// hipGraph captured once per key on a library-owned stream and replayed on
// the context's stream.
template <typename F>
int run_maybe_graph(mpm_ctx *c, mpm_ctx::GraphSlot &slot,
                    const mpm_ctx::GraphKey &key, F &&body) {
  // (re-binning synchronises with the host: never captured)
  if (!c->use_graphs || c->prof.mask || c->tape.T == 0 || c->tape.rebin) return body();
  if (!slot.valid || !(slot.key == key)) {
    if (slot.exec) (void)hipGraphExecDestroy(slot.exec);
    slot.exec = nullptr;
    slot.valid = false;
    if (!c->cap_stream)
      RC(hip_ok(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking)));
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    hipGraph_t g = nullptr;
    int rc = hip_ok(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    if (!rc) {
      const int rb = body();
      const hipError_t e = hipStreamEndCapture(c->stream, &g);
      rc = rb ? rb : hip_ok(e);
    }
    c->stream = user;
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    rc = hip_ok(hipGraphInstantiate(&slot.exec, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    if (rc) return rc;
    slot.key = key;
    slot.valid = true;
  }
  return hip_ok(hipGraphLaunch(slot.exec, c->stream));
}

mpm_ctx::GraphKey graph_key(mpm_ctx *c) {
  mpm_ctx::GraphKey k;
  const auto &t = c->tape;
  k.T = t.T;
  k.k = t.k;
  k.memo = t.memo;
  k.grids_all = t.grids_all;
  k.sorted = t.sorted;
  int nch = 0;
  k.p[6] = cur_chunks(c, &nch);
  k.nch = nch;
  k.nne = bin(c).n_ne;
  k.p[0] = t.states;
  k.p[1] = t.grids;
  k.p[2] = t.act;
  k.p[3] = t.pp;
  k.p[4] = t.adj;
  k.p[5] = c->gact;
  k.p[7] = c->ctl.on ? c->ctl.Z : nullptr;
  k.ctl = c->ctl.on ? c->ctl.nz : 0;
  k.rev = t.rev ? 2 * t.rev + t.rev_spine : 0;
  k.mat = c->has_mat;
  return k;
}

// ---- binomial checkpointing ------------------------------------------------
// Reversing L substeps from a held state with c further state slots: either
// recompute every state from the held one (c = 0: L (L - 1) / 2 substeps) or
// advance m substeps, store that state, reverse the last L - m substeps with
// c - 1 slots and then the first m with c slots.  The fewest substeps this
// takes is the binomial count of Griewank's checkpointing analysis,
//   F(L, c) = t L - beta(c + 2, t - 1),  t = min{t : beta(c + 1, t) >= L},
//   beta(c, t) = (c + t)! / (c! t!),
// and the split taken is the first m that attains it.

int64_t rev_beta(int64_t c, int64_t t) {
  if (t < 0) return 0;
  // C(c + t, t) with saturation (the values compared against are < 2^62)
  double b = 1.0;
  for (int64_t i = 1; i <= t; ++i) {
    b = b * (double)(c + i) / (double)i;
    if (b > 4.0e18) return (int64_t)4e18;
  }
  return (int64_t)std::llround(b);
}

int64_t rev_cost(int64_t L, int64_t c) {
  if (L <= 1) return 0;
  if (c <= 0) return L * (L - 1) / 2;
  int64_t t = 0;
  while (rev_beta(c + 1, t) < L) ++t;
  return t * L - rev_beta(c + 2, t - 1);
}

int64_t rev_split(int64_t L, int64_t c) {
  const int64_t best = rev_cost(L, c);
  for (int64_t m = 1; m < L; ++m)
    if (m + rev_cost(L - m, c - 1) + rev_cost(m, c) == best) return m;
  return L / 2;  // not reached when the closed form holds
}

// Forward substep n of a rollout: state `in` -> state `out` (must differ).
int fwd_substep(mpm_ctx *c, int n, const State &in, const State &out) {
  int nch = 0;
  const Chunk *chunks = cur_chunks(c, &nch);
  const bool tiles = c->tape.sorted;
  const float *act = c->n_act ? c->tape.act + (int64_t)n * c->n_act : nullptr;
  RC(fwd_p2g(c, tiles, chunks, nch, cs(in), cur_act_id(c), act, c->gm, c->gp, n));
  RC(fwd_grid(c, tiles, c->gm, c->gp, c->gv, 1));
  return fwd_g2p(c, chunks, nch, cs(in), out, c->gv, nullptr, nullptr, nullptr, false, n);
}

int ctl_forward(mpm_ctx *c, const State &s, int n, int g2p_rows = 0);
int ctl_adjoint(mpm_ctx *c, int n, const double *sbar, const State &g);

// Binomial tapes: slot 0 = S^0, slots 1..rev = checkpoints, slot rev + 1 =
// work state, slot rev + 2 = S^T.  The forward sweep stores the checkpoints
// of the reverse schedule's first descent (its rightmost path).
int rollout_forward_revolve(mpm_ctx *c, int T) {
  const int64_t sf = c->state_floats();
  const int R = c->tape.rev;
  std::vector<int> slot_at((size_t)T + 1, -1);
  int64_t lo = 0, cf = R;
  int slot = 0;
  while (T - lo > 1 && cf > 0) {
    lo += rev_split(T - lo, cf);
    slot_at[(size_t)lo] = ++slot;
    --cf;
  }
  float *cur = slot_state(c, 0);
  for (int n = 0; n < T; ++n) {
    float *dst = n + 1 == T ? slot_state(c, R + 2)
                 : slot_at[(size_t)n + 1] >= 0 ? slot_state(c, slot_at[(size_t)n + 1])
                 : c->tape.pp + (int64_t)((n + 1) & 1) * sf;
    if (c->ctl.on) RC(ctl_forward(c, state_at(c, cur), n));
    RC(fwd_substep(c, n, state_at(c, cur), state_at(c, dst)));
    cur = dst;
  }
  return MPM_OK;
}

// Reverse pass of a binomial tape.  A0/A1: the adjoint ping-pong pair (the
// adjoint of S^T in A1 on entry).
struct RevolveRun {
  mpm_ctx *c;
  State A0, A1;
  int nga;

  // S^{n0} in `src` -> S^{n1} in `dst` (n1 > n0), intermediates in the tape's
  // ping-pong pair
  int advance(float *src, int n0, int n1, float *dst) {
    const int64_t sf = c->state_floats();
    for (int n = n0; n < n1; ++n) {
      float *in = n == n0 ? src : c->tape.pp + (int64_t)((n - n0) & 1) * sf;
      float *out = n + 1 == n1 ? dst : c->tape.pp + (int64_t)((n + 1 - n0) & 1) * sf;
      RC(fwd_substep(c, n, state_at(c, in), state_at(c, out)));
    }
    return MPM_OK;
  }
  // adjoint of substep n from S^n: the grid of step n is recomputed first
  int leaf(int n, float *sbuf) {
    int nch = 0;
    const Chunk *chunks = cur_chunks(c, &nch);
    const bool tiles = c->tape.sorted;
    const State s = state_at(c, sbuf);
    const float *act = c->n_act ? c->tape.act + (int64_t)n * c->n_act : nullptr;
    float *g = slot_grid(c, 0);
    RC(fwd_p2g(c, tiles, chunks, nch, cs(s), cur_act_id(c), act, c->gm, c->gp, n));
    RC(fwd_grid(c, tiles, c->gm, c->gp, c->gv, 1, g, g + c->G));
    double *ga = nga ? c->gact + (int64_t)n * c->n_act : nullptr;
    RC(bwd_step(c, tiles, chunks, nch, cs(s), cur_act_id(c), act, g, g + c->G,
                cs(A1), A0, ga, n));
    if (c->ctl.on) RC(ctl_adjoint(c, n, ga, A0));
    std::swap(A0, A1);
    return MPM_OK;
  }
  // reverse substeps [lo, hi) from S^lo in slot `slot`, cf free slots above
  // it; `stored`: the first-descent checkpoints are already in place
  int run(int lo, int hi, int64_t cf, int slot, bool stored) {
    const int L = hi - lo;
    if (L == 1) return leaf(lo, slot_state(c, slot));
    if (cf == 0) {
      float *work = slot_state(c, c->tape.rev + 1);
      for (int n = hi - 1; n >= lo; --n) {
        float *sb = slot_state(c, slot);
        if (n > lo) {
          RC(advance(sb, lo, n, work));
          sb = work;
        }
        RC(leaf(n, sb));
      }
      return MPM_OK;
    }
    const int m = lo + (int)rev_split(L, cf);
    if (!stored) RC(advance(slot_state(c, slot), lo, m, slot_state(c, slot + 1)));
    RC(run(m, hi, cf - 1, slot + 1, stored));
    return run(lo, m, cf, slot, false);
  }
};

// Controller at substep n: component means of state n -> z^n (tape) ->
// a^n = tanh(W z^n + b) into the tape's actuation row n.  g2p_rows > 0: the
// G2P that produced state n already wrote that many rows of component sums
// (only the reduction runs).
int ctl_forward(mpm_ctx *c, const State &s, int n, int g2p_rows) {
  const auto &k = c->ctl;
  CtlArgs a;
  a.dim = c->dim;
  a.N = (int)c->N;
  a.n_comp = k.n_comp;
  a.n_act = c->n_act;
  a.nz = k.nz;
  a.comp = k.comp;
  a.inv_cnt = k.inv_cnt;
  a.x = s.x;
  a.v = s.v;
  a.ld = (int)c->N;
  a.partial = k.partial;
  a.sums = k.sums;
  a.done = k.done;
  a.W = k.W;
  a.b = k.b;
  a.target = k.target;
  a.act = c->tape.act + (int64_t)n * c->n_act;
  a.z = k.Z + (int64_t)n * k.nz;
  if (g2p_rows > 0) return launch_ctl_reduce(a, g2p_rows, c->stream) ? MPM_ERR_HIP : MPM_OK;
  return launch_ctl_forward(a, c->stream) ? MPM_ERR_HIP : MPM_OK;
}

// Reverse of the controller at substep n: adds its term to the adjoint of
// state n (g) and to dL/dW, dL/db; sbar = dL/ds^n from the substep's reverse.
int ctl_adjoint(mpm_ctx *c, int n, const double *sbar, const State &g) {
  const auto &k = c->ctl;
  CtlAdjArgs a;
  a.dim = c->dim;
  a.N = (int)c->N;
  a.n_comp = k.n_comp;
  a.n_act = c->n_act;
  a.nz = k.nz;
  a.comp = k.comp;
  a.inv_cnt = k.inv_cnt;
  a.W = k.W;
  a.act = c->tape.act + (int64_t)n * c->n_act;
  a.z = k.Z + (int64_t)n * k.nz;
  a.sbar = sbar;
  a.gW = k.gW;
  a.gb = k.gb;
  a.gx = g.x;
  a.gv = g.v;
  a.ld = (int)c->N;
  return launch_ctl_adjoint(a, c->stream) ? MPM_ERR_HIP : MPM_OK;
}

// Binning sets 1 .. n-1 for re-binned tapes (allocated once, kept).
int ensure_bins(mpm_ctx *c, int n) {
  const int64_t N = std::max<int64_t>(c->N, 1), nt = c->n_tiles;
  while ((int)c->bins.size() < n) {
    BinSet b;
    b.owned = true;
    RC(dmalloc(&b.tile_cnt, nt, c->stream));
    RC(dmalloc(&b.tile_start, nt + 1, c->stream));
    RC(dmalloc(&b.perm, N, c->stream));
    RC(dmalloc(&b.act, N, c->stream));
    RC(dmalloc(&b.tile_list, nt, c->stream));
    RC(dmalloc(&b.pscene, N, c->stream));
    RC(dmalloc(&b.rel, N, c->stream));
    RC(dmalloc(&b.chunks, N / CH + nt + 1, c->stream));
    if (c->use_nt && c->dim == 3) RC(dmalloc(&b.nt_cand, (int64_t)c->n_nt * 8, c->stream));
    c->bins.push_back(b);
  }
  return MPM_OK;
}

// Re-binning into binning j: `slot` holds a checkpoint state in binning
// j-1's order; binning j is computed from its positions and the state is put
// into the new order in place (through the scratch state).
int rebin_at(mpm_ctx *c, int j, float *slot) {
  BinSet &dst = c->bins[(size_t)j];
  RC(bin_particles(c, state_at(c, slot).x, dst, &c->bins[(size_t)j - 1]));
  const State tmp = state_at(c, c->scratch);
  RC(permute_state_by(c, ms(state_at(c, slot)), tmp, dst.rel, 0));
  RC(copy_state(c, ms(tmp), state_at(c, slot)));
  c->cur_bin = j;
  c->n_bins = j + 1;
  return MPM_OK;
}

// Adaptive re-binning (rebin = 2): at a checkpoint, the particles that the
// last segment's scatters sent beyond their tile box's slack (global
// atomics) are read back; past 0.5% of the segment's particle-substeps the
// particles are binned again.  The count restarts at every checkpoint.
constexpr double REBIN_OVERFLOW = 0.005;
int overflow_wants_rebin(mpm_ctx *c, int seg_len, bool *want) {
  RC(hip_ok(hipMemcpyAsync(c->h_over, c->d_over, sizeof(int), hipMemcpyDeviceToHost,
                           c->stream)));
  RC(hip_ok(hipStreamSynchronize(c->stream)));
  *want = (double)*c->h_over > REBIN_OVERFLOW * (double)c->N * (double)seg_len;
  return launch_fill_i32(c->d_over, 1, c->stream);
}

int rollout_forward(mpm_ctx *c, const Layout &L) {
  if (c->tape.rev) return rollout_forward_revolve(c, L.T);
  int nch = 0;
  const Chunk *chunks = cur_chunks(c, &nch);
  const int *ids = cur_act_id(c);
  const bool tiles = c->tape.sorted;
  const bool rebin = c->tape.rebin != 0;
  // 3D binned rollouts with the sorted scatter fuse each G2P with the next
  // substep's P2G (state n+1 goes from registers to the scatter)
  // (not with a closed-loop controller: the actuation of substep n+1 needs
  // the component means of state n+1 first)
  // (not in deterministic mode: there G2P is the same kernel as the
  // reverse pass's recompute)
  const bool fuse = tiles && c->scatter_mode == 3 && c->dim == 3 && !c->ctl.on &&
                    c->fuse_forward && !c->det;
  auto act_of = [&](int n) {
    return c->n_act ? c->tape.act + (int64_t)n * c->n_act : nullptr;
  };
  if (rebin) c->tape.seg_bin.assign((size_t)((L.T + L.k - 1) / L.k), 0);
  if (c->tape.rebin == 2) RC(launch_fill_i32(c->d_over, 1, c->stream));
  for (int n = 0; n < L.T; ++n) {
    // re-binned tapes: a checkpoint starts a new binning (every one, or
    // where the last segment's particles overflowed their tile boxes)
    bool new_bin = false;
    if (rebin && n > 0 && n % L.k == 0) {
      new_bin = true;
      if (c->tape.rebin == 2) RC(overflow_wants_rebin(c, L.k, &new_bin));
      if (new_bin) {
        RC(rebin_at(c, c->n_bins, fwd_slot(c, L, n)));
        chunks = cur_chunks(c, &nch);
        ids = cur_act_id(c);
      }
      c->tape.seg_bin[(size_t)(n / L.k)] = c->n_bins - 1;
    }
    const State s = state_at(c, fwd_slot(c, L, n));
    const State o = state_at(c, fwd_slot(c, L, n + 1));
    // the controller's component sums of state n come from the G2P that
    // produced it (substep 0: their own kernel)
    if (c->ctl.on) RC(ctl_forward(c, s, n, n > 0 ? nch : 0));
    // (on re-binned tapes the G2P before a checkpoint runs unfused, whether
    // or not the checkpoint changes the binning)
    if (!fuse || n == 0 || (rebin && n % L.k == 0))
      RC(fwd_p2g(c, tiles, chunks, nch, cs(s), ids, act_of(n), c->gm, c->gp, n));
    if (c->tape.grids_all) {
      float *g = slot_grid(c, n);  // keep this substep's grid on the tape
      RC(fwd_grid(c, tiles, c->gm, c->gp, c->gv, 1, g, g + c->G));
    } else {
      RC(fwd_grid(c, tiles, c->gm, c->gp, c->gv, 1));
    }
    if (fuse && n + 1 < L.T && !(rebin && (n + 1) % L.k == 0)) {
      // (a checkpoint of a re-binned tape may change the order: P2G there
      // runs after the decision)
      // state n+1 is read back only through x and F unless the tape keeps
      // it (memo, or a checkpoint)
      RC(fwd_g2p_p2g(c, cs(s), o, c->gv, ids, act_of(n + 1),
                     L.memo || (n + 1) % L.k == 0 || keeps_last_segment(c, L, n + 1), n));
    } else if (c->det && c->tape.grids_all) {
      // deterministic mode: the velocities are rebuilt from the stored
      // (m, p) exactly as the reverse pass's recompute does, so a
      // checkpointed reverse pass sees the forward pass's states bit for bit
      const float *g = slot_grid(c, n);
      RC(fwd_g2p(c, chunks, nch, cs(s), o, nullptr, g, g + c->G, nullptr,
                 c->ctl.on && n + 1 < L.T, n));
    } else {
      RC(fwd_g2p(c, chunks, nch, cs(s), o, c->gv, nullptr, nullptr, nullptr,
                 c->ctl.on && n + 1 < L.T, n));
    }
  }
  return MPM_OK;
}

// Reverse pass over library-owned buffers only: reads the adjoint of S^T
// from adj slot 0, leaves the adjoint of S^0 in adj slot adj_out_slot(c).
// (one swap of the two adjoint slots per substep and, on re-binned tapes,
// one per change of binning)
int adj_out_slot(const mpm_ctx *c) {
  const auto &t = c->tape;
  return (t.T + (t.rebin ? c->n_bins - 1 : 0)) & 1;
}

int rollout_backward_core(mpm_ctx *c) {
  auto &t = c->tape;
  const Layout L{t.T, t.k, t.memo, t.memo ? t.T + 1 : (t.T + t.k - 1) / t.k + 1};
  int nch = 0;
  const Chunk *chunks = cur_chunks(c, &nch);
  const int *ids = cur_act_id(c);
  const bool tiles = t.sorted;
  const int64_t sf = c->state_floats();
  State A1 = state_at(c, t.adj), A0 = state_at(c, t.adj + sf);
  // step calls may have left their grid in gm/gp; recomputed P2Gs start at 0
  RC(launch_fill_f32(c->gm, c->G, c->stream));
  RC(launch_fill_f32(c->gp, c->dim * c->G, c->stream));
  const int64_t nga = (int64_t)t.T * c->n_act;
  if (nga > 0) RC(launch_fill_f64(c->gact, nga, c->stream));
  if (c->has_mat) RC(launch_fill_f32(c->gmat, 3 * c->N, c->stream));
  if (c->ctl.on) {
    RC(launch_fill_f64(c->ctl.gW, (int64_t)c->n_act * c->ctl.nz, c->stream));
    RC(launch_fill_f64(c->ctl.gb, c->n_act, c->stream));
  }
  if (t.rev) {
    // A1 holds the adjoint of S^T (adj slot 0): the first leaf reads it.
    // The schedule overwrites the first-descent checkpoints; a later reverse
    // pass over the same tape advances them again from S^0.
    RevolveRun r{c, A0, A1, nga > 0 ? 1 : 0};
    return t.T > 0 ? r.run(0, t.T, t.rev, 0, t.rev_spine != 0) : MPM_OK;
  }
  // (a memo tape is one segment whose states are all stored)
  const int nseg = t.memo ? (t.T > 0 ? 1 : 0) : (t.T + t.k - 1) / t.k;
  const int seglen = t.memo ? t.T : t.k;
  const bool keep = !t.memo && t.grids_all;  // stored grids: G2P-only recompute
  // 3D binned reverse passes fuse each gather with the previous substep's
  // scatter (not with a closed-loop controller, whose adjoint adds to the
  // state adjoint between the two, nor with a per-particle material field)
  const bool fuse = tiles && c->scatter_mode == 3 && c->dim == 3 && !c->ctl.on &&
                    !c->has_mat && c->fuse_reverse;
  // state n of segment j (segment states alternate between two banks when
  // the grids are kept, so one segment can be recomputed while the adjoint
  // of the next one runs; the last segment's states, kept by the forward
  // pass, are in a third bank)
  auto S = [&](int j, int n) -> float * {
    const int n0 = j * seglen;
    if (t.memo) return slot_state(c, n);
    if (n == n0) return slot_state(c, j);
    const int64_t bank = keep ? (j == nseg - 1 ? 2 : (j & 1)) : 0;
    return slot_state(c, L.ncp + bank * t.k + (n - n0));
  };
  auto Gr = [&](int n0, int n) -> float * {
    return t.grids_all ? slot_grid(c, n) : slot_grid(c, n - n0);
  };
  // re-binned tapes: segment j's states are in binning seg_bin[j]'s order
  auto seg_chunks = [&](int j, int *n) -> const Chunk * {
    if (!t.rebin) return cur_chunks(c, n);
    const BinSet &b = c->bins[(size_t)t.seg_bin[(size_t)j]];
    *n = b.n_chunks;
    return b.chunks;
  };
  // recompute segment j's states from its checkpoint with G2P alone,
  // reading each substep's stored grid
  auto recompute = [&](int j, hipStream_t st) -> int {
    if (j == nseg - 1) return MPM_OK;  // kept by the forward pass
    const int n0 = j * seglen, n1 = std::min(t.T, n0 + seglen);
    int nc = 0;
    const Chunk *ch = seg_chunks(j, &nc);
    for (int n = n0; n + 1 < n1; ++n) {
      const float *g = Gr(n0, n);
      RC(fwd_g2p(c, ch, nc, cs(state_at(c, S(j, n))), state_at(c, S(j, n + 1)),
                 nullptr, g, g + c->G, st, false, n));
    }
    return MPM_OK;
  };
  // overlap: the recompute of segment j-1 runs on a second stream while the
  // adjoint kernels of segment j run on the context's stream (not under
  // graph capture, nor while G2P launches are being timed)
  const bool overlap = keep && nseg > 1 && !(c->use_graphs && !c->prof.mask) &&
                       !((c->prof.mask >> MPM_K_G2P) & 1u);
  if (overlap) {
    if (!c->aux_stream)
      RC(hip_ok(hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking)));
    for (hipEvent_t *e : {&c->ev_start, &c->ev_recomp, &c->ev_adj})
      if (!*e) RC(hip_ok(hipEventCreateWithFlags(e, hipEventDisableTiming)));
    RC(hip_ok(hipEventRecord(c->ev_start, c->stream)));
    RC(hip_ok(hipStreamWaitEvent(c->aux_stream, c->ev_start, 0)));
    RC(recompute(nseg - 1, c->aux_stream));
    RC(hip_ok(hipEventRecord(c->ev_recomp, c->aux_stream)));
  }
  for (int j = nseg - 1; j >= 0; --j) {
    const int n0 = j * seglen, n1 = std::min(t.T, n0 + seglen);
    if (t.rebin) {
      c->cur_bin = t.seg_bin[(size_t)j];
      chunks = cur_chunks(c, &nch);
      ids = cur_act_id(c);
    }
    if (overlap) {
      // segment j's states are ready; start segment j-1's recompute once the
      // adjoint of segment j+1 (same bank) is done
      RC(hip_ok(hipStreamWaitEvent(c->stream, c->ev_recomp, 0)));
      if (j > 0) {
        RC(hip_ok(hipStreamWaitEvent(c->aux_stream, c->ev_adj, 0)));
        RC(recompute(j - 1, c->aux_stream));
        RC(hip_ok(hipEventRecord(c->ev_recomp, c->aux_stream)));
      }
    } else if (keep) {
      RC(recompute(j, nullptr));
    } else if (!t.memo) {
      // recompute the segment from its checkpoint, keeping states and grids
      for (int n = n0; n < n1; ++n) {
        const State s = state_at(c, S(j, n));
        const float *act = c->n_act ? t.act + (int64_t)n * c->n_act : nullptr;
        float *g = Gr(n0, n);
        RC(fwd_p2g(c, tiles, chunks, nch, cs(s), ids, act, c->gm, c->gp, n));
        RC(fwd_grid(c, tiles, c->gm, c->gp, c->gv, 1, g, g + c->G));
        if (n + 1 < n1)
          RC(fwd_g2p(c, chunks, nch, cs(s), state_at(c, S(j, n + 1)), c->gv, nullptr,
                     nullptr, nullptr, false, n));
      }
    }
    auto act_of = [&](int n) {
      return c->n_act ? t.act + (int64_t)n * c->n_act : nullptr;
    };
    auto gact_of = [&](int n) {
      return nga > 0 ? c->gact + (int64_t)n * c->n_act : nullptr;
    };
    if (fuse && n1 - n0 >= 2) {
      // scatter and grid reverse of the segment's last substep, then per
      // substep the gather fused with the previous substep's scatter, then
      // the first substep's gather
      const float *g = Gr(n0, n1 - 1);
      RC(bwd_scatter(c, tiles, chunks, nch, cs(state_at(c, S(j, n1 - 1))), cs(A1), n1 - 1));
      RC(bwd_grid(c, tiles, g, g + c->G));
      for (int n = n1 - 1; n > n0; --n) {
        RC(bwd_gather_scatter(c, cs(state_at(c, S(j, n))), cs(state_at(c, S(j, n - 1))),
                              ids, act_of(n), cs(A1), A0, gact_of(n), n));
        std::swap(A0, A1);
        const float *gp = Gr(n0, n - 1);
        RC(bwd_grid(c, tiles, gp, gp + c->G));
      }
      RC(bwd_gather(c, tiles, chunks, nch, cs(state_at(c, S(j, n0))), ids, act_of(n0),
                    cs(A1), A0, gact_of(n0), n0));
      std::swap(A0, A1);
    } else {
      for (int n = n1 - 1; n >= n0; --n) {
        const State s = state_at(c, S(j, n));
        const float *g = Gr(n0, n);
        RC(bwd_step(c, tiles, chunks, nch, cs(s), ids, act_of(n), g, g + c->G, cs(A1),
                    A0, gact_of(n), n));
        // a^n = tanh(W z(S^n) + b): its dependence on state n
        if (c->ctl.on) RC(ctl_adjoint(c, n, c->gact + (int64_t)n * c->n_act, A0));
        std::swap(A0, A1);
      }
    }
    if (t.rebin && j > 0 && t.seg_bin[(size_t)j] != t.seg_bin[(size_t)j - 1]) {
      // the adjoint of S^{n0} from segment j's binning into the one before
      RC(permute_state_by(c, ms(A1), A0, c->bins[(size_t)t.seg_bin[(size_t)j]].rel, 1));
      std::swap(A0, A1);
    }
    if (overlap) RC(hip_ok(hipEventRecord(c->ev_adj, c->stream)));
  }
  return MPM_OK;
}

int rollout_backward(mpm_ctx *c, const mpm_state *gT, mpm_state *g0,
                     float *g_act, float *g_W = nullptr, float *g_b = nullptr) {
  auto &t = c->tape;
  const int64_t sf = c->state_floats();
  const State A_in = state_at(c, t.adj);
  // the seed is put into the order of the last binning of the tape
  if (t.rebin) c->cur_bin = c->n_bins - 1;
  if (t.sorted) RC(permute_state(c, *gT, A_in, 0));
  else RC(copy_state(c, *gT, A_in));
  const int64_t nga = (int64_t)t.T * c->n_act;
  if (nga > 0) RC(ensure_gact(c, nga));
  RC(run_maybe_graph(c, c->gbwd, graph_key(c), [&] { return rollout_backward_core(c); }));
  t.rev_spine = 0;  // (outside the captured body: replays skip the body)
  c->gmat_sorted = t.sorted;
  c->gmat_valid = c->has_mat;
  c->cur_bin = 0;
  const State A_out = state_at(c, t.adj + adj_out_slot(c) * sf);
  if (t.sorted) RC(permute_state(c, ms(A_out), st(*g0), 1));
  else RC(copy_state(c, ms(A_out), st(*g0)));
  if (g_act && nga > 0)
    RC(launch_gact_store(c->gact, g_act, nga, 0, c->stream));
  if (c->ctl.on && g_W)
    RC(launch_gact_store(c->ctl.gW, g_W, (int64_t)c->n_act * c->ctl.nz, 0, c->stream));
  if (c->ctl.on && g_b)
    RC(launch_gact_store(c->ctl.gb, g_b, c->n_act, 0, c->stream));
  return MPM_OK;
}

}  // namespace

extern "C" {

const char *mpm_strerror(int code) {
  switch (code) {
    case MPM_OK: return "ok";
    case MPM_ERR_ARG: return "invalid argument";
    case MPM_ERR_OOM: return "out of device memory";
    case MPM_ERR_DOMAIN: return "particle stencil outside the grid";
    case MPM_ERR_INVERTED: return "deformation gradient with det F <= 0";
    case MPM_ERR_NONFINITE: return "non-finite value produced";
    case MPM_ERR_HIP: return "HIP runtime error";
    case MPM_ERR_STATE: return "call out of order (no tape)";
    default: return "unknown error";
  }
}

void mpm_destroy(mpm_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  dfree(c->d_over, c->stream);
  if (c->h_over) (void)hipHostFree(c->h_over);
  dfree(c->d_scenes, c->stream);
  dfree(c->d_chunks_user, c->stream);
  dfree(c->d_gblocks, c->stream);
  dfree(c->d_act_id, c->stream);
  dfree(c->d_pscene, c->stream);
  dfree(c->gm, c->stream);
  dfree(c->gp, c->stream);
  dfree(c->gv, c->stream);
  dfree(c->vbar, c->stream);
  dfree(c->pbar, c->stream);
  dfree(c->mbar, c->stream);
  dfree(c->gact, c->stream);
  dfree(c->d_err, c->stream);
  dfree(c->scratch, c->stream);
  dfree(c->d_tile_scene, c->stream);
  dfree(c->d_tile_cnt, c->stream);
  dfree(c->d_cell_cnt, c->stream);
  dfree(c->d_ptile, c->stream);
  dfree(c->d_pcell, c->stream);
  dfree(c->d_prank, c->stream);
  dfree(c->d_tile_start, c->stream);
  dfree(c->d_nch, c->stream);
  dfree(c->d_chunk_start, c->stream);
  dfree(c->d_perm, c->stream);
  dfree(c->d_act_sorted, c->stream);
  dfree(c->d_chunks_sorted, c->stream);
  dfree(c->d_part, c->stream);
  dfree(c->mat_user, c->stream);
  dfree(c->mat_sorted, c->stream);
  dfree(c->gmat, c->stream);
  dfree(c->ctl.comp, c->stream);
  dfree(c->ctl.inv_cnt, c->stream);
  dfree(c->ctl.W, c->stream);
  dfree(c->ctl.b, c->stream);
  dfree(c->ctl.target, c->stream);
  dfree(c->ctl.partial, c->stream);
  dfree(c->ctl.sums, c->stream);
  dfree(c->ctl.done, c->stream);
  dfree(c->ctl.gW, c->stream);
  dfree(c->ctl.gb, c->stream);
  dfree(c->ctl.Z, c->stream);
  dfree(c->d_tile_flag, c->stream);
  dfree(c->d_tile_pos, c->stream);
  dfree(c->d_tile_list, c->stream);
  for (auto &b : c->bins) {
    dfree(b.pscene, c->stream);
    dfree(b.nt_cand, c->stream);
    if (!b.owned) continue;
    dfree(b.tile_cnt, c->stream);
    dfree(b.tile_start, c->stream);
    dfree(b.perm, c->stream);
    dfree(b.act, c->stream);
    dfree(b.tile_list, c->stream);
    dfree(b.rel, c->stream);
    dfree(b.chunks, c->stream);
  }
  c->bins.clear();
  dfree(c->d_nt_scene, c->stream);
  dfree(c->d_nt_dirty, c->stream);
  dfree(c->d_cell_start, c->stream);
  dfree(c->d_cell_list, c->stream);
  dfree(c->sb_part, c->stream);
  dfree(c->d_act_scene, c->stream);
  dfree(c->tape.states, c->stream);
  dfree(c->tape.grids, c->stream);
  dfree(c->tape.act, c->stream);
  dfree(c->tape.pp, c->stream);
  dfree(c->tape.adj, c->stream);
  for (hipEvent_t e : c->prof.pool) (void)hipEventDestroy(e);
  if (c->gfwd.exec) (void)hipGraphExecDestroy(c->gfwd.exec);
  if (c->gbwd.exec) (void)hipGraphExecDestroy(c->gbwd.exec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->aux_stream) (void)hipStreamDestroy(c->aux_stream);
  for (hipEvent_t e : {c->ev_start, c->ev_recomp, c->ev_adj})
    if (e) (void)hipEventDestroy(e);
  delete c;
}

int mpm_init(mpm_ctx **out, const mpm_scene *scenes, int n_scenes,
             const int32_t *act_id, void *stream, const mpm_opts *opts) {
  if (!out) return MPM_ERR_ARG;
  *out = nullptr;
  if (!scenes || n_scenes <= 0) return MPM_ERR_ARG;
  const int dim = scenes[0].dim;
  if (dim != 2 && dim != 3) return MPM_ERR_ARG;
  int tile = dim == 2 ? 8 : 4;
  int sort = 1;
  int scatter = 0;
  int recompute_grids = 0;
  int graphs = 0;
  int fusion = 0;
  int det = 0;
  int persistent = 0;
  int rebin = 0;
  if (opts) {
    for (int k = 0; k < 1; ++k)
      if (opts->reserved[k]) return MPM_ERR_ARG;
    if (opts->persistent != 0 && opts->persistent != 1) return MPM_ERR_ARG;
    persistent = opts->persistent;
    if (opts->rebin < 0 || opts->rebin > 2) return MPM_ERR_ARG;
    rebin = opts->rebin;
    if (opts->fusion < 0 || opts->fusion > 2) return MPM_ERR_ARG;
    fusion = opts->fusion;
    if (opts->deterministic != 0 && opts->deterministic != 1) return MPM_ERR_ARG;
    det = opts->deterministic;
    if (opts->graphs != 0 && opts->graphs != 1) return MPM_ERR_ARG;
    graphs = opts->graphs;
    if (opts->recompute_grids != 0 && opts->recompute_grids != 1) return MPM_ERR_ARG;
    recompute_grids = opts->recompute_grids;
    if (opts->scatter < 0 || opts->scatter > 3) return MPM_ERR_ARG;
    scatter = opts->scatter;
    if (opts->tile && !tile_supported(dim, opts->tile)) return MPM_ERR_ARG;
    if (opts->tile) tile = opts->tile;
    if (opts->sort != 0 && opts->sort != 1) return MPM_ERR_ARG;
    sort = opts->sort;
  }
  int64_t N = 0, G = 0, n_tiles = 0;
  int n_act = 0;
  for (int s = 0; s < n_scenes; ++s) {
    const mpm_scene &S = scenes[s];
    if (!scene_valid(S, dim)) return MPM_ERR_ARG;
    const int64_t nn = dim == 2 ? (int64_t)S.n_grid * S.n_grid
                                : (int64_t)S.n_grid * S.n_grid * S.n_grid;
    const int64_t nt1 = (S.n_grid - 2 + tile - 1) / tile;
    N += S.n_particles;
    G += nn;
    n_act += S.n_act;
    n_tiles += dim == 2 ? nt1 * nt1 : nt1 * nt1 * nt1;
  }
  if (N > (int64_t)INT32_MAX / 16 || G > (int64_t)INT32_MAX / 4 ||
      n_tiles > (int64_t)INT32_MAX / 4096)
    return MPM_ERR_ARG;

  mpm_ctx *c = new mpm_ctx();
  c->dim = dim;
  c->n_scenes = n_scenes;
  c->N = N;
  c->G = G;
  c->n_act = n_act;
  c->tile = tile;
  c->sort = sort;
  c->keep_grids = !recompute_grids;
  c->use_graphs = graphs;
  c->persistent = persistent;
  c->rebin = rebin;
  c->fuse_forward = fusion != 1;
  c->fuse_reverse = fusion == 2;
  {
    const int cells = dim == 2 ? tile * tile : tile * tile * tile;
    if ((scatter == 2 || scatter == 3) && cells != 64) {
      delete c;
      return MPM_ERR_ARG;
    }
    c->scatter_mode = scatter == 0 ? (cells == 64 ? 3 : 1) : scatter;
    // deterministic sums need the binned, sorted scatter
    if (det && (!sort || c->scatter_mode != 3)) {
      delete c;
      return MPM_ERR_ARG;
    }
    c->det = det;
  }
  c->stream = (hipStream_t)stream;
  c->n_tiles = (int)n_tiles;

  std::vector<Chunk> chunks;
  std::vector<GridBlock> gblocks;
  std::vector<int> pscene(N), tile_scene, nt_scene;
  int64_t ntoff = 0;
  c->h_act_id.assign(N, -1);
  int64_t poff = 0, goff = 0, toff = 0;
  int aoff = 0;
  for (int s = 0; s < n_scenes; ++s) {
    const mpm_scene &S = scenes[s];
    DevScene d = dev_scene(S, tile);
    d.p_off = (int)poff;
    d.g_off = (int)goff;
    d.act_off = aoff;
    d.tile_off = (int)toff;
    d.nt_off = (int)ntoff;
    {
      const int64_t nnts = dim == 2 ? (int64_t)d.nnt * d.nnt : (int64_t)d.nnt * d.nnt * d.nnt;
      for (int64_t k = 0; k < nnts; ++k) nt_scene.push_back(s);
      ntoff += nnts;
    }
    c->h_scenes.push_back(d);
    for (int64_t k = 0; k < S.n_particles; k += CH) {
      Chunk ch{s, (int)(poff + k), (int)std::min<int64_t>(CH, S.n_particles - k), 0};
      chunks.push_back(ch);
    }
    const int64_t nn = dim == 2 ? (int64_t)S.n_grid * S.n_grid
                                : (int64_t)S.n_grid * S.n_grid * S.n_grid;
    for (int64_t k = 0; k < nn; k += 256) {
      GridBlock gb{s, (int)k, (int)std::min<int64_t>(256, nn - k), 0};
      gblocks.push_back(gb);
    }
    for (int64_t p = 0; p < S.n_particles; ++p) {
      pscene[poff + p] = s;
      if (act_id) {
        const int j = act_id[poff + p];
        if (j < -1 || j >= S.n_act) {
          delete c;
          return MPM_ERR_ARG;
        }
        c->h_act_id[poff + p] = j;
      }
    }
    const int64_t nt1 = (S.n_grid - 2 + tile - 1) / tile;
    const int64_t nts = dim == 2 ? nt1 * nt1 : nt1 * nt1 * nt1;
    for (int64_t k = 0; k < nts; ++k) tile_scene.push_back(s);
    poff += S.n_particles;
    goff += nn;
    toff += nts;
    aoff += S.n_act;
  }
  c->n_chunks_user = (int)chunks.size();
  c->n_gblocks = (int)gblocks.size();
  const int64_t cpt = dim == 2 ? tile * tile : tile * tile * tile;

  int rc = MPM_OK;
#define TRY(x)                      \
  do {                              \
    rc = (x);                       \
    if (rc) {                       \
      mpm_destroy(c);               \
      return rc;                    \
    }                               \
  } while (0)
  TRY(dmalloc(&c->d_scenes, n_scenes, c->stream));
  TRY(dmalloc(&c->d_chunks_user, c->n_chunks_user, c->stream));
  TRY(dmalloc(&c->d_gblocks, c->n_gblocks, c->stream));
  TRY(dmalloc(&c->d_act_id, N, c->stream));
  TRY(dmalloc(&c->d_pscene, N, c->stream));
  TRY(dmalloc(&c->gm, G, c->stream));
  TRY(dmalloc(&c->gp, dim * G, c->stream));
  TRY(dmalloc(&c->gv, dim * G, c->stream));
  TRY(dmalloc(&c->vbar, dim * G, c->stream));
  TRY(dmalloc(&c->pbar, dim * G, c->stream));
  TRY(dmalloc(&c->mbar, G, c->stream));
  TRY(dmalloc(&c->d_err, 1, c->stream));
  TRY(dmalloc(&c->scratch, c->state_floats(), c->stream));
  TRY(dmalloc(&c->d_tile_scene, n_tiles, c->stream));
  TRY(dmalloc(&c->d_tile_cnt, n_tiles, c->stream));
  TRY(dmalloc(&c->d_cell_cnt, n_tiles * cpt, c->stream));
  TRY(dmalloc(&c->d_ptile, N, c->stream));
  TRY(dmalloc(&c->d_pcell, N, c->stream));
  TRY(dmalloc(&c->d_prank, N, c->stream));
  TRY(dmalloc(&c->d_tile_start, n_tiles + 1, c->stream));
  TRY(dmalloc(&c->d_nch, n_tiles, c->stream));
  TRY(dmalloc(&c->d_chunk_start, n_tiles + 1, c->stream));
  TRY(dmalloc(&c->d_perm, N, c->stream));
  TRY(dmalloc(&c->d_act_sorted, N, c->stream));
  TRY(dmalloc(&c->d_chunks_sorted, N / CH + n_tiles + 1, c->stream));
  TRY(dmalloc(&c->d_tile_flag, n_tiles, c->stream));
  TRY(dmalloc(&c->d_tile_pos, n_tiles + 1, c->stream));
  TRY(dmalloc(&c->d_tile_list, n_tiles, c->stream));
  {
    BinSet b0;
    b0.tile_cnt = c->d_tile_cnt;
    b0.tile_start = c->d_tile_start;
    b0.perm = c->d_perm;
    b0.act = c->d_act_sorted;
    b0.tile_list = c->d_tile_list;
    b0.chunks = c->d_chunks_sorted;
    if (c->rebin) TRY(dmalloc(&b0.pscene, std::max<int64_t>(N, 1), c->stream));
    c->bins.assign(1, b0);
  }
  if (c->rebin == 2) {
    TRY(dmalloc(&c->d_over, 1, c->stream));
    TRY(hip_ok(hipHostMalloc((void **)&c->h_over, sizeof(int), hipHostMallocDefault)));
  }
  c->n_nt = (int)ntoff;
  c->use_nt = c->scatter_mode == 3 && c->n_nt > 0;
  if (c->use_nt) {
    TRY(dmalloc(&c->d_nt_scene, c->n_nt, c->stream));
    TRY(dmalloc(&c->d_nt_dirty, c->n_nt, c->stream));
    if (c->dim == 3) TRY(dmalloc(&c->bins[0].nt_cand, (int64_t)c->n_nt * 8, c->stream));
  }
  if (c->det) {
    TRY(dmalloc(&c->d_cell_start, n_tiles * cpt + 1, c->stream));
    TRY(dmalloc(&c->d_cell_list, std::max<int64_t>(N, 1), c->stream));
    TRY(dmalloc(&c->sb_part, std::max<int64_t>(N, 1), c->stream));
    if (n_act > 0) TRY(dmalloc(&c->d_act_scene, n_act, c->stream));
  }
  {
    const int64_t S = tile + 4;
    TRY(dmalloc(&c->d_part, n_tiles * (dim + 1) * (dim == 2 ? S * S : S * S * S), c->stream));
  }
  if (n_act > 0) TRY(ensure_gact(c, n_act));

  hipStream_t s = c->stream;
  TRY(hip_ok(hipMemcpyAsync(c->d_scenes, c->h_scenes.data(),
                            sizeof(DevScene) * n_scenes, hipMemcpyHostToDevice, s)));
  TRY(hip_ok(hipMemcpyAsync(c->d_chunks_user, chunks.data(),
                            sizeof(Chunk) * chunks.size(), hipMemcpyHostToDevice, s)));
  TRY(hip_ok(hipMemcpyAsync(c->d_gblocks, gblocks.data(),
                            sizeof(GridBlock) * gblocks.size(), hipMemcpyHostToDevice, s)));
  if (N > 0) {
    TRY(hip_ok(hipMemcpyAsync(c->d_act_id, c->h_act_id.data(), sizeof(int) * N,
                              hipMemcpyHostToDevice, s)));
    TRY(hip_ok(hipMemcpyAsync(c->d_pscene, pscene.data(), sizeof(int) * N,
                              hipMemcpyHostToDevice, s)));
  }
  TRY(hip_ok(hipMemcpyAsync(c->d_tile_scene, tile_scene.data(),
                            sizeof(int) * tile_scene.size(), hipMemcpyHostToDevice, s)));
  if (c->use_nt) {
    TRY(hip_ok(hipMemcpyAsync(c->d_nt_scene, nt_scene.data(), sizeof(int) * c->n_nt,
                              hipMemcpyHostToDevice, s)));
    TRY(launch_fill_i32(c->d_nt_dirty, c->n_nt, s));
  }
  std::vector<int> act_scene;
  if (c->det && n_act > 0) {
    for (int sc_i = 0; sc_i < n_scenes; ++sc_i)
      for (int j = 0; j < scenes[sc_i].n_act; ++j) act_scene.push_back(sc_i);
    TRY(hip_ok(hipMemcpyAsync(c->d_act_scene, act_scene.data(), sizeof(int) * n_act,
                              hipMemcpyHostToDevice, s)));
  }
  TRY(launch_fill_f32(c->gm, G, s));
  TRY(launch_fill_f32(c->gp, dim * G, s));
  TRY(launch_fill_f32(c->gv, dim * G, s));
  TRY(launch_fill_f32(c->vbar, dim * G, s));
  TRY(launch_fill_f32(c->pbar, dim * G, s));
  TRY(launch_fill_f32(c->mbar, G, s));
  TRY(launch_fill_i32((int *)c->d_err, 1, s));
  TRY(hip_ok(hipStreamSynchronize(s)));
#undef TRY
  *out = c;
  return MPM_OK;
}

int mpm_set_stream(mpm_ctx *c, void *stream) {
  if (!c) return MPM_ERR_ARG;
  c->stream = (hipStream_t)stream;
  return MPM_OK;
}

int mpm_tape_generation(const mpm_ctx *c, uint64_t *gen) {
  if (!c || !gen) return MPM_ERR_ARG;
  *gen = c->tape_gen;
  return MPM_OK;
}

int mpm_tape_binnings(const mpm_ctx *c, int32_t *n) {
  if (!c || !n) return MPM_ERR_ARG;
  *n = c->n_bins;
  return MPM_OK;
}

int mpm_info(const mpm_ctx *c, int64_t *n_particles, int32_t *n_act,
             int64_t *n_nodes) {
  if (!c) return MPM_ERR_ARG;
  if (n_particles) *n_particles = c->N;
  if (n_act) *n_act = c->n_act;
  if (n_nodes) *n_nodes = c->G;
  return MPM_OK;
}

int mpm_sync_errors(mpm_ctx *c) {
  if (!c) return MPM_ERR_ARG;
  if (c->poisoned) return c->poisoned;
  return read_err(c);
}

int mpm_step_forward(mpm_ctx *c, const mpm_state *s_n, const float *act_n,
                     mpm_state *s_np1) {
  RC(check_ctx(c));
  if (!state_ok(c, s_n) || !state_ok(c, s_np1) || (c->n_act && !act_n))
    return MPM_ERR_ARG;
  RC(launch_fill_f32(c->gm, c->G, c->stream));
  RC(launch_fill_f32(c->gp, c->dim * c->G, c->stream));
  RC(fwd_p2g(c, false, c->d_chunks_user, c->n_chunks_user, cs(*s_n),
             c->d_act_id, act_n, c->gm, c->gp));
  RC(fwd_grid(c, false, c->gm, c->gp, c->gv, 0));
  RC(fwd_g2p(c, c->d_chunks_user, c->n_chunks_user, cs(*s_n), st(*s_np1),
             c->gv));
  return MPM_OK;
}

}  // extern "C"

// ---- allocation-free single substep -----------------------------------------
// Device memory of mpm_step_forward_noalloc: one static region per GPU (each
// device holds its own copy, at its own address, until the process ends).
// Layout: scene descriptor, chunks, node blocks, sanitised actuator ids, grid
// m, p, v of at most MPM_NOALLOC_MAX_NODES nodes.
namespace {
constexpr int64_t NA_SCENE = 0;
constexpr int64_t NA_CHUNKS = 256;
constexpr int64_t NA_BLOCKS = NA_CHUNKS + sizeof(Chunk) * (MPM_NOALLOC_MAX_PARTICLES / CH);
constexpr int64_t NA_ACT = NA_BLOCKS + sizeof(GridBlock) * (MPM_NOALLOC_MAX_NODES / 256);
constexpr int64_t NA_GRID = NA_ACT + sizeof(int) * MPM_NOALLOC_MAX_PARTICLES;
constexpr int64_t NA_BYTES = NA_GRID + sizeof(float) * 7 * MPM_NOALLOC_MAX_NODES;
static_assert(NA_BLOCKS % 256 == 0 && NA_ACT % 256 == 0 && NA_GRID % 256 == 0,
              "regions keep 256-byte alignment");
static_assert(sizeof(DevScene) <= 256, "the scene descriptor fits its slot");
}  // namespace

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {
constexpr int NA_MAX_DEVICES = 64;
std::mutex na_mutex;
unsigned char *na_ptr[NA_MAX_DEVICES] = {};

// The device address of `scratch` on the current device (looked up once per
// device; host code never uses the array's name as an address).
int noalloc_region(unsigned char **out) {
  int dev = 0;
  RC(hip_ok(hipGetDevice(&dev)));
  if (dev < 0 || dev >= NA_MAX_DEVICES) return MPM_ERR_ARG;
  std::lock_guard<std::mutex> lock(na_mutex);
  if (!na_ptr[dev]) {
    void *p = nullptr;
    RC(hip_ok(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))));
    if (!p) return MPM_ERR_HIP;
    na_ptr[dev] = static_cast<unsigned char *>(p);
  }
  *out = na_ptr[dev];
  return MPM_OK;
}
}  // namespace

extern "C" {

int mpm_step_forward_noalloc(const mpm_scene *scene, const int32_t *act_id,
                             const mpm_state *s_n, const float *act_n,
                             mpm_state *s_np1, uint32_t *err, void *stream) {
  if (!scene || !s_n || !s_np1 || !err) return MPM_ERR_ARG;
  const int dim = scene->dim;
  if ((dim != 2 && dim != 3) || !scene_valid(*scene, dim)) return MPM_ERR_ARG;
  const int64_t n = scene->n_grid;
  const int64_t nodes = dim == 2 ? n * n : n * n * n;
  const int64_t N = scene->n_particles;
  if (nodes > MPM_NOALLOC_MAX_NODES || N > MPM_NOALLOC_MAX_PARTICLES) return MPM_ERR_ARG;
  if (scene->n_act > 0 && !act_n) return MPM_ERR_ARG;
  if (N > 0 && (!s_n->x || !s_n->v || !s_n->C || !s_n->F || !s_np1->x || !s_np1->v ||
                !s_np1->C || !s_np1->F))
    return MPM_ERR_ARG;
  unsigned char *base = nullptr;
  RC(noalloc_region(&base));
  hipStream_t st = (hipStream_t)stream;
  DevScene *d_sc = reinterpret_cast<DevScene *>(base + NA_SCENE);
  Chunk *chunks = reinterpret_cast<Chunk *>(base + NA_CHUNKS);
  GridBlock *blocks = reinterpret_cast<GridBlock *>(base + NA_BLOCKS);
  int *ids = reinterpret_cast<int *>(base + NA_ACT);
  float *gm = reinterpret_cast<float *>(base + NA_GRID);
  float *gp = gm + MPM_NOALLOC_MAX_NODES;
  float *gv = gp + 3 * MPM_NOALLOC_MAX_NODES;
  const int64_t G = MPM_NOALLOC_MAX_NODES;  // plane stride of p and v
  unsigned *d_err = reinterpret_cast<unsigned *>(err);

  NoAllocArgs na;
  na.sc = dev_scene(*scene, dim == 2 ? 8 : 4);
  na.dim = dim;
  na.N = (int)N;
  na.nodes = nodes;
  na.G = G;
  na.scene = d_sc;
  na.chunks = chunks;
  na.blocks = blocks;
  na.act_id_in = act_id;
  na.act_id = ids;
  na.gm = gm;
  na.gp = gp;
  na.err = d_err;
  if (launch_noalloc_setup(na, st)) return MPM_ERR_HIP;

  const CState s{s_n->x, s_n->v, s_n->C, s_n->F};
  const State o{s_np1->x, s_np1->v, s_np1->C, s_np1->F};
  P2GArgs a1{};
  a1.scenes = d_sc;
  a1.chunks = chunks;
  a1.n_chunks = (int)((N + CH - 1) / CH);
  a1.s = s;
  a1.ld = (int)N;
  a1.act_id = ids;
  a1.act = act_n;
  a1.gm = gm;
  a1.gp = gp;
  a1.G = G;
  a1.err = d_err;
  if (launch_p2g(dim, a1, st)) return MPM_ERR_HIP;
  GridArgs a2{};
  a2.scenes = d_sc;
  a2.blocks = blocks;
  a2.n_blocks = (int)((nodes + 255) / 256);
  a2.gm = gm;
  a2.gp = gp;
  a2.gv = gv;
  a2.G = G;
  a2.zero_mp = 0;  // the next call clears m and p in its set-up
  if (launch_grid(dim, a2, st)) return MPM_ERR_HIP;
  G2PArgs a3{};
  a3.scenes = d_sc;
  a3.chunks = chunks;
  a3.n_chunks = a1.n_chunks;
  a3.s = s;
  a3.out = o;
  a3.ld = (int)N;
  a3.gv = gv;
  a3.G = G;
  a3.err = d_err;
  if (launch_g2p(dim, a3, st)) return MPM_ERR_HIP;
  return MPM_OK;
}

int mpm_get_grid(mpm_ctx *c, float *m, float *p, float *v) {
  if (!c) return MPM_ERR_ARG;
  const size_t g = sizeof(float) * c->G;
  if (m) RC(hip_ok(hipMemcpyAsync(m, c->gm, g, hipMemcpyDeviceToDevice, c->stream)));
  if (p)
    RC(hip_ok(hipMemcpyAsync(p, c->gp, g * c->dim, hipMemcpyDeviceToDevice, c->stream)));
  if (v)
    RC(hip_ok(hipMemcpyAsync(v, c->gv, g * c->dim, hipMemcpyDeviceToDevice, c->stream)));
  return MPM_OK;
}

int mpm_step_backward(mpm_ctx *c, const mpm_state *s_n, const float *act_n,
                      const mpm_state *g_np1, mpm_state *g_n, float *g_act_n) {
  RC(check_ctx(c));
  if (!state_ok(c, s_n) || !state_ok(c, g_np1) || !state_ok(c, g_n) ||
      (c->n_act && !act_n))
    return MPM_ERR_ARG;
  // forward grid of step n (the adjoint gather rebuilds C of state n+1
  // from it)
  RC(launch_fill_f32(c->gm, c->G, c->stream));
  RC(launch_fill_f32(c->gp, c->dim * c->G, c->stream));
  RC(fwd_p2g(c, false, c->d_chunks_user, c->n_chunks_user, cs(*s_n),
             c->d_act_id, act_n, c->gm, c->gp));
  RC(fwd_grid(c, false, c->gm, c->gp, c->gv, 0));
  double *gact = nullptr;
  if (g_act_n && c->n_act > 0) {
    RC(ensure_gact(c, c->n_act));
    RC(launch_fill_f64(c->gact, c->n_act, c->stream));
    gact = c->gact;
  }
  if (c->has_mat) RC(launch_fill_f32(c->gmat, 3 * c->N, c->stream));
  RC(bwd_step(c, false, c->d_chunks_user, c->n_chunks_user, cs(*s_n),
              c->d_act_id, act_n, c->gm, c->gp, cs(*g_np1), st(*g_n), gact));
  if (gact) RC(launch_gact_store(gact, g_act_n, c->n_act, 1, c->stream));
  c->gmat_sorted = 0;
  c->gmat_valid = c->has_mat;
  return MPM_OK;
}

int mpm_set_horizons(mpm_ctx *c, const int32_t *t_end) {
  RC(check_ctx(c));
  if (t_end)
    for (int s = 0; s < c->n_scenes; ++s)
      if (t_end[s] < 0) return MPM_ERR_ARG;
  ++c->tape_gen;
  c->tape.valid = 0;  // a tape recorded under other horizons is not reversed
  for (int s = 0; s < c->n_scenes; ++s) c->h_scenes[s].t_end = t_end ? t_end[s] : INT32_MAX;
  c->horizons = false;
  for (int s = 0; s < c->n_scenes; ++s) c->horizons = c->horizons || c->h_scenes[s].t_end != INT32_MAX;
  return hip_ok(hipMemcpyAsync(c->d_scenes, c->h_scenes.data(),
                               sizeof(DevScene) * c->n_scenes, hipMemcpyHostToDevice,
                               c->stream));
}

int mpm_set_materials(mpm_ctx *c, const float *E_p, const float *rho_p) {
  RC(check_ctx(c));
  ++c->tape_gen;
  c->gmat_valid = 0;
  if (!E_p && !rho_p) {
    c->has_mat = 0;
    return MPM_OK;
  }
  if (c->N == 0) return MPM_OK;
  hipStream_t s = c->stream;
  if (!c->mat_user) {
    RC(dmalloc(&c->mat_user, 3 * c->N, s));
    RC(dmalloc(&c->mat_sorted, 3 * c->N, s));
    RC(dmalloc(&c->gmat, 3 * c->N, s));
  }
  RC(launch_mat_field(c->d_scenes, c->d_pscene, (int)c->N, E_p, rho_p, c->mat_user, s));
  // a tape already binned reads its materials in its own order
  if (c->tape.valid && c->tape.sorted)
    RC(launch_permute_rows(c->mat_user, c->mat_sorted, c->d_perm, (int)c->N,
                           (int)c->N, 3, 0, s));
  c->has_mat = 1;
  return MPM_OK;
}

int mpm_material_grad(mpm_ctx *c, float *g_E, float *g_rho) {
  RC(check_ctx(c));
  if (!c->has_mat || !c->gmat_valid) return MPM_ERR_STATE;
  if (c->N == 0) return MPM_OK;
  return launch_mat_grad(c->d_scenes, c->d_pscene, (int)c->N,
                         c->gmat_sorted ? c->d_perm : nullptr, c->gmat, g_E, g_rho,
                         c->stream);
}

}  // extern "C"

namespace {

// Controller set-up for a rollout of T substeps: checks the component ids
// (on the host), copies W, b, target into library buffers and the ids into
// the tape's particle order (after binning).
int ctl_setup(mpm_ctx *c, const mpm_controller *u, int T) {
  auto &k = c->ctl;
  const int d = c->dim, N = (int)c->N;
  std::vector<int32_t> h((size_t)N);
  RC(hip_ok(hipMemcpyAsync(h.data(), u->comp_id, sizeof(int32_t) * N,
                           hipMemcpyDeviceToHost, c->stream)));
  RC(hip_ok(hipStreamSynchronize(c->stream)));
  std::vector<int64_t> cnt((size_t)u->n_comp, 0);
  for (int p = 0; p < N; ++p) {
    const int q = h[(size_t)p];
    if (q < -1 || q >= u->n_comp) return MPM_ERR_ARG;
    if (q >= 0) ++cnt[(size_t)q];
  }
  float inv[CTL_MAX_COMP] = {};
  for (int q = 0; q < u->n_comp; ++q) {
    if (cnt[(size_t)q] == 0) return MPM_ERR_ARG;  // a mean over no particle
    inv[q] = (float)(1.0 / (double)cnt[(size_t)q]);
  }
  hipStream_t s = c->stream;
  if (!k.comp) {
    RC(dmalloc(&k.comp, c->N, s));
    RC(dmalloc(&k.inv_cnt, CTL_MAX_COMP, s));
    RC(dmalloc(&k.W, (int64_t)CTL_MAX_ACT * CTL_MAX_NZ, s));
    RC(dmalloc(&k.b, CTL_MAX_ACT, s));
    RC(dmalloc(&k.target, 3, s));
    RC(dmalloc(&k.sums, CTL_MAX_ZS, s));
    RC(dmalloc(&k.done, 1, s));
    RC(launch_fill_i32((int *)k.done, 1, s));
    RC(dmalloc(&k.gW, (int64_t)CTL_MAX_ACT * CTL_MAX_NZ, s));
    RC(dmalloc(&k.gb, CTL_MAX_ACT, s));
  }
  // rows of component sums: one per workgroup of the controller's own sum
  // kernel, or one per G2P chunk (the G2P of each substep writes them)
  {
    int nch = 0;
    (void)cur_chunks(c, &nch);
    const int rows = std::max(ctl_rows(N), nch);
    if (rows > k.partial_rows) {
      dfree(k.partial, s);
      k.partial_rows = 0;
      RC(dmalloc(&k.partial, (int64_t)rows * CTL_MAX_ZS, s));
      k.partial_rows = rows;
    }
  }
  k.n_comp = u->n_comp;
  k.nz = d * (1 + 2 * u->n_comp);
  if ((int64_t)T * k.nz > k.Z_cap) {
    dfree(k.Z, s);
    k.Z_cap = 0;
    RC(dmalloc(&k.Z, (int64_t)T * k.nz, s));
    k.Z_cap = (int64_t)T * k.nz;
  }
  RC(hip_ok(hipMemcpyAsync(k.inv_cnt, inv, sizeof(inv), hipMemcpyHostToDevice, s)));
  RC(hip_ok(hipMemcpyAsync(k.W, u->W, sizeof(float) * c->n_act * k.nz,
                           hipMemcpyDeviceToDevice, s)));
  RC(hip_ok(hipMemcpyAsync(k.b, u->b, sizeof(float) * c->n_act,
                           hipMemcpyDeviceToDevice, s)));
  RC(hip_ok(hipMemcpyAsync(k.target, u->target, sizeof(float) * d,
                           hipMemcpyDeviceToDevice, s)));
  if (c->tape.sorted)
    RC(launch_permute_i32(u->comp_id, k.comp, c->d_perm, N, s));
  else
    RC(hip_ok(hipMemcpyAsync(k.comp, u->comp_id, sizeof(int32_t) * N,
                             hipMemcpyDeviceToDevice, s)));
  RC(hip_ok(hipStreamSynchronize(s)));  // `inv` is host memory
  k.on = 1;
  return MPM_OK;
}

// Body shared by the open-loop and closed-loop rollouts (arguments checked).
int rollout_run(mpm_ctx *c, int T, int ckpt_k, const mpm_state *s0,
                const float *act, const mpm_controller *ctl, mpm_state *sT) {
  auto &t = c->tape;
  ++c->tape_gen;
  t.valid = 0;
  t.rev_spine = 0;
  c->ctl.on = 0;
  const int rev = ckpt_k < 0 ? -ckpt_k : 0;
  const int memo = ckpt_k == 0;
  const int k = memo || rev ? 1 : std::min(ckpt_k, std::max(T, 1));
  const int ncp = rev ? rev + 3 : memo ? T + 1 : (T + k - 1) / k + 1;
  const int grids_all = !rev && (memo || c->keep_grids);
  // checkpointed tapes with stored grids keep three banks of segment
  // states: two for the reverse pass, which recomputes one segment while it
  // runs the adjoint of the next, and one for the last segment, kept by the
  // forward pass; binomial tapes hold rev + 3 states and one grid
  const int64_t nstates = rev ? ncp : memo ? T + 1 : ncp + (grids_all ? 3 * k : k);
  const int64_t ngrids = rev ? 1 : grids_all ? T : k;
  RC(ensure_tape(c, nstates, ngrids, (int64_t)T * c->n_act));
  t.T = T;
  t.k = k;
  t.memo = memo;
  t.rev = rev;
  t.grids_all = grids_all;
  t.sorted = c->sort && c->N > 0;
  // re-binning at every checkpoint: checkpointed tapes of binned rollouts
  // without a controller (its component sums follow one order) or a
  // per-particle material field (sorted once per tape)
  t.rebin = c->rebin && t.sorted && !memo && !rev && k < T && !ctl && !c->has_mat ? c->rebin : 0;
  if (t.rebin) RC(ensure_bins(c, (T + k - 1) / k));
  if (!ctl && c->n_act && T > 0)
    RC(hip_ok(hipMemcpyAsync(t.act, act, sizeof(float) * T * c->n_act,
                             hipMemcpyDeviceToDevice, c->stream)));
  const Layout L{T, k, memo, ncp};
  const State S0 = state_at(c, slot_state(c, 0));
  c->cur_bin = 0;
  c->n_bins = 1;
  if (t.sorted) {
    RC(bin_particles(c, s0->x, c->bins[0]));
    RC(permute_state(c, *s0, S0, 0));
  } else {
    RC(copy_state(c, *s0, S0));
  }
  if (ctl) RC(ctl_setup(c, ctl, T));
  // the step calls leave their grid in gm/gp; rollouts start from zero
  RC(launch_fill_f32(c->gm, c->G, c->stream));
  RC(launch_fill_f32(c->gp, c->dim * c->G, c->stream));
  RC(run_maybe_graph(c, c->gfwd, graph_key(c), [&] { return rollout_forward(c, L); }));
  const State ST = state_at(c, fwd_slot(c, L, T));
  if (t.sorted) RC(permute_state(c, ms(ST), st(*sT), 1));
  else RC(copy_state(c, ms(ST), st(*sT)));
  t.rev_spine = rev ? 1 : 0;
  t.valid = 1;
  return MPM_OK;
}

}  // namespace

extern "C" {

int64_t mpm_revolve_steps(int64_t L, int32_t slots) {
  if (L < 0 || slots < 0) return -1;
  return rev_cost(L, slots);
}

int64_t mpm_revolve_split(int64_t L, int32_t slots) {
  if (L < 2 || slots < 1) return -1;
  return rev_split(L, slots);
}

int mpm_rollout(mpm_ctx *c, int T, int ckpt_k, const mpm_state *s0,
                const float *act, mpm_state *sT, const mpm_state *gT,
                mpm_state *g0, float *g_act) {
  RC(check_ctx(c));
  if (T < 0 || ckpt_k < -MPM_MAX_REVOLVE_SLOTS || !state_ok(c, s0) || !state_ok(c, sT) ||
      (c->n_act && T > 0 && !act) || (gT && !state_ok(c, gT)) ||
      (gT && !state_ok(c, g0)))
    return MPM_ERR_ARG;
  RC(rollout_run(c, T, ckpt_k, s0, act, nullptr, sT));
  if (gT) return rollout_backward(c, gT, g0, g_act);
  return MPM_OK;
}

int mpm_rollout_ctrl(mpm_ctx *c, int T, int ckpt_k, const mpm_state *s0,
                     const mpm_controller *ctl, mpm_state *sT, float *act,
                     const mpm_state *gT, mpm_state *g0, float *g_act,
                     float *g_W, float *g_b) {
  RC(check_ctx(c));
  if (T < 0 || ckpt_k < -MPM_MAX_REVOLVE_SLOTS || !state_ok(c, s0) || !state_ok(c, sT) || !ctl ||
      (gT && !state_ok(c, gT)) || (gT && !state_ok(c, g0)))
    return MPM_ERR_ARG;
  if (c->n_scenes != 1 || c->N < 1 || c->n_act < 1 || c->n_act > CTL_MAX_ACT ||
      ctl->n_comp < 1 || 2 * c->dim * ctl->n_comp > CTL_MAX_ZS || !ctl->comp_id ||
      !ctl->W || !ctl->b || !ctl->target || c->horizons)
    return MPM_ERR_ARG;
  RC(rollout_run(c, T, ckpt_k, s0, nullptr, ctl, sT));
  if (act && T > 0)
    RC(hip_ok(hipMemcpyAsync(act, c->tape.act, sizeof(float) * T * c->n_act,
                             hipMemcpyDeviceToDevice, c->stream)));
  if (gT) return rollout_backward(c, gT, g0, g_act, g_W, g_b);
  return MPM_OK;
}

int mpm_rollout_ctrl_backward(mpm_ctx *c, const mpm_state *gT, mpm_state *g0,
                              float *g_act, float *g_W, float *g_b) {
  RC(check_ctx(c));
  if (!c->tape.valid || !c->ctl.on) return MPM_ERR_STATE;
  if (!state_ok(c, gT) || !state_ok(c, g0)) return MPM_ERR_ARG;
  return rollout_backward(c, gT, g0, g_act, g_W, g_b);
}

int mpm_rollout_backward(mpm_ctx *c, const mpm_state *gT, mpm_state *g0,
                         float *g_act) {
  RC(check_ctx(c));
  if (!c->tape.valid) return MPM_ERR_STATE;
  if (!state_ok(c, gT) || !state_ok(c, g0)) return MPM_ERR_ARG;
  return rollout_backward(c, gT, g0, g_act);
}

int mpm_profile(mpm_ctx *c, uint32_t mask) {
  if (!c || (mask >> MPM_NUM_KERNELS)) return MPM_ERR_ARG;
  c->prof.mask = mask;
  return MPM_OK;
}

int mpm_profile_read(mpm_ctx *c, int64_t *count, double *ms) {
  if (!c) return MPM_ERR_ARG;
  auto &P = c->prof;
  RC(hip_ok(hipStreamSynchronize(c->stream)));
  for (size_t i = 0; i < P.kid.size(); ++i) {
    float t = 0.0f;
    RC(hip_ok(hipEventElapsedTime(&t, P.pool[2 * i], P.pool[2 * i + 1])));
    P.count[P.kid[i]] += 1;
    P.ms[P.kid[i]] += t;
  }
  for (int k = 0; k < MPM_NUM_KERNELS; ++k) {
    if (count) count[k] = P.count[k];
    if (ms) ms[k] = P.ms[k];
    P.count[k] = 0;
    P.ms[k] = 0.0;
  }
  P.kid.clear();
  P.used = 0;
  return MPM_OK;
}

int mpm_act_bank_forward(void *stream, int T, int n_act, int n_freq, float dt,
                         const float *freq, const float *amp,
                         const float *phase, float *act) {
  if (T < 0 || n_act < 0 || n_freq < 0) return MPM_ERR_ARG;
  if ((int64_t)T * n_act == 0) return MPM_OK;
  if (!act || (n_freq > 0 && (!freq || !amp || !phase))) return MPM_ERR_ARG;
  return launch_act_bank_fwd(T, n_act, n_freq, dt, freq, amp, phase, act,
                             (hipStream_t)stream);
}

int mpm_act_bank_backward(void *stream, int T, int n_act, int n_freq,
                          float dt, const float *freq, const float *amp,
                          const float *phase, const float *g_act,
                          float *g_amp, float *g_phase) {
  if (T < 0 || n_act < 0 || n_freq < 0) return MPM_ERR_ARG;
  if (n_act * n_freq == 0) return MPM_OK;
  if (!freq || !amp || !phase || !g_amp || !g_phase || (T > 0 && !g_act))
    return MPM_ERR_ARG;
  return launch_act_bank_bwd(T, n_act, n_freq, dt, freq, amp, phase, g_act,
                             g_amp, g_phase, (hipStream_t)stream);
}

}  // extern "C"
