// mpm_internal.h -- device-side data structures shared by the gfx950 kernels
// (mpm_kernels.hip) and the host implementation of the C ABI (mpm_api.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpm {

// Particles handled by one workgroup (one particle per lane, 4 waves).
constexpr int CH = 256;
// Largest bounding box of grid nodes a workgroup stages in LDS; chunks whose
// stencil box is larger fall back to global atomics / global loads.
constexpr int LDS_NODES = 1024;
// Per-scene actuators reduced in LDS by the adjoint gather; scenes with more
// actuators add straight to global memory.
constexpr int LDS_ACT = 64;

// Sticky device error bits (ORed into the context's error word).
enum : unsigned { EB_DOMAIN = 1u, EB_INVERTED = 2u, EB_NONFINITE = 4u,
                  EB_ACT_ID = 8u /* allocation-free step: actuator id out of range */ };

// Per-scene constants, precomputed on the host in FP32.
struct DevScene {
  int n;        // nodes per axis
  int np;       // particles of the scene
  int p_off;    // first particle (in the concatenated arrays)
  int g_off;    // first grid node (in the concatenated grids)
  int n_act;    // actuators of the scene
  int act_off;  // first actuator (in the concatenated actuation vector)
  int wall;     // sticky-wall thickness in nodes
  int tile_off; // first tile of the scene (binning)
  int nt;       // tiles per axis (binning)
  int bc;       // wall nodes: 0 sticky, 1 friction projection
  float fric;   // friction coefficient (bc = 1)
  float nu;     // Poisson ratio (per-particle Lame parameters from E_p)
  float dt, dx, inv_dx, Dinv;  // Dinv = 4 / dx^2
  float mu, la, mp, V0;        // Lame parameters, particle mass and volume
  float kG;                    // -Dinv * dt * V0 (stress part of G_p)
  int nnt;      // node tiles per axis (binning; node tile t: nodes tB-1 .. tB+B-2)
  int nt_off;   // first node tile of the scene
  int t_end;    // the scene is held fixed from substep t_end on (its horizon)
  float g[3];                  // gravity
  float axis[3];               // actuation axis
};

// A run of consecutive particles handled by one workgroup.
struct Chunk {
  int scene, start, count, pad;
};

// A run of consecutive grid nodes of one scene handled by one workgroup.
struct GridBlock {
  int scene, start, count, pad;
};

// Particle state (or its adjoint) in structure-of-arrays layout with leading
// dimension ld: component a of particle p at a*ld + p.
struct State {
  float *x, *v, *C, *F;
};
struct CState {
  const float *x, *v, *C, *F;
};

// ---------------------------------------------------------------------------
// kernel launchers (mpm_kernels.hip)
// ---------------------------------------------------------------------------

// Tiles of binned particles.  A tile owns the particles whose stencil base
// lies in a B^d block of cells; its workgroup accumulates their scatter into
// an LDS box of S^d nodes (S = B + 4: the block, the 2-node stencil reach and
// one cell of drift on every side) and stores the whole box, so the grid
// kernels can sum the (at most 2 per axis) boxes covering each node without
// global atomics.  Particles that drifted further add to the grid directly.
template <int B>
struct TileBox {
  static constexpr int S = B + 4;
};

struct TileInfo {
  const int *cnt;    // particles per tile [n_tiles]
  const int *start;  // first (sorted) particle of each tile
  const int *scene;  // scene of each tile
  float *part;       // partial boxes [n_tiles][d+1][S^d]
  int B;             // cells per tile edge
  const int *list;   // non-null: workgroup b handles tile list[b] (non-empty tiles)
  int *nt_dirty;     // non-null: node tiles that particles beyond their box's slack
                     // reached with global atomics (set to 1, per rollout)
  int *n_over = nullptr;  // non-null: particles scattered with global atomics
                          // (beyond their box's slack) are counted here
};

struct P2GArgs {
  const DevScene *scenes;
  const Chunk *chunks;
  int n_chunks;
  CState s;
  int ld;
  const int *act_id;  // scene-local actuator of each particle (-1 passive)
  const float *act;   // [n_act_tot] for this step
  float *gm, *gp;     // grid mass [G], momentum [d][G]
  int64_t G;
  unsigned *err;
  TileInfo tiles;     // tile path only
  const float *mat = nullptr;  // per-particle (mu, la, m_p) [3][ld] or null
  int det = 0;       // deterministic sums (fixed order of a cell's records)
  int n = 0;         // substep index (scenes past their horizon are held fixed)
};

struct GridArgs {
  const DevScene *scenes;
  const GridBlock *blocks;
  int n_blocks;
  float *gm, *gp, *gv;
  int64_t G;
  int zero_mp;  // clear m and p after reading them (next P2G starts at 0)
  const int *tile_cnt;  // non-null: add the tile boxes in `part`
  const float *part;
  int B;
  float *out_m, *out_p;  // non-null: store the summed m and p here (may be gm/gp)
  // node-tile launch (binned rollouts, 64-cell tiles): one wave per node
  // tile, nt_scene: scene of each node tile, nt_dirty: see TileInfo
  const int *nt_scene = nullptr;
  const int *nt_dirty = nullptr;
  int n_nt = 0;  int persist = 0;  // persistent launch: a few workgroups loop over the node tiles
  // 3D, 4^3-cell tiles: per node tile the 8 covering tiles that hold
  // particles (-1 for none), built at binning ([n_nt][8]; null: from counts)
  const int *nt_cand = nullptr;
};

struct G2PArgs {
  const DevScene *scenes;
  const Chunk *chunks;
  int n_chunks;
  CState s;     // reads x, F
  State out;    // writes x, v, C, F (may alias s)
  int ld;
  const float *gv;
  const float *gm, *gp;  // non-null: velocities from these m, p (not gv)
  int64_t G;
  unsigned *err;
  // non-null: the controller's per-chunk component sums of the new state
  // into ctl_partial (entry-major, ctl_rows >= n_chunks rows)
  const int *ctl_comp = nullptr;
  float *ctl_partial = nullptr;
  int ctl_nzs = 0, ctl_rows = 0;
  int n = 0;         // substep index (scenes past their horizon are held fixed)
};

// G2P of substep n fused with the binned P2G of substep n+1 (3D rollouts):
// reads x, F of state n and the grid velocity of substep n, writes state
// n+1, scatters state n+1 into the tile boxes (and the overflow grid gm, gp).
struct G2P2GArgs {
  const DevScene *scenes;
  CState s;           // state n (x, F read)
  State out;          // state n+1 (x, F written; v, C too when write_vc); must not alias s
  int ld;
  int write_vc;       // state n+1 is kept on the tape: write v and C too
  const float *gv;    // grid velocity of substep n
  const int *act_id;  // scene-local actuator of each particle (-1 passive)
  const float *act;   // [n_act_tot] of substep n+1
  float *gm, *gp;     // overflow grid of substep n+1
  int64_t G;
  unsigned *err;
  TileInfo tiles;
  const float *mat = nullptr;  // per-particle (mu, la, m_p) [3][ld] or null
  int det = 0;       // deterministic sums (fixed order of a cell's records)
  int n = 0;         // substep index (scenes past their horizon are held fixed)
};

struct AdjScatterArgs {
  const DevScene *scenes;
  const Chunk *chunks;
  int n_chunks;
  CState s;     // state n: x, F
  CState g1;    // adjoint of state n+1
  int ld;
  float *vbar;  // [d][G] accumulated
  int64_t G;
  unsigned *err;
  TileInfo tiles;  // tile path only
  int det = 0;       // deterministic sums (fixed order of a cell's records)
  int n = 0;         // substep index (scenes past their horizon are held fixed)
};

struct AdjGridArgs {
  const DevScene *scenes;
  const GridBlock *blocks;
  int n_blocks;
  const float *gm, *gp;  // forward grid of step n
  float *vbar;           // read, then cleared
  float *pbar, *mbar, *gv;  // written: dL/dp, dL/dm, forward v
  int64_t G;
  const int *tile_cnt;  // non-null: add the tile boxes in `part` to vbar
  const float *part;
  int B;
  const int *nt_scene = nullptr;  // node-tile launch (see GridArgs)
  const int *nt_dirty = nullptr;
  int n_nt = 0;  int persist = 0;  // persistent launch: a few workgroups loop over the node tiles
  const int *nt_cand = nullptr;    // see GridArgs
};

struct AdjGatherArgs {
  const DevScene *scenes;
  const Chunk *chunks;
  int n_chunks;
  CState s;          // state n
  CState g1;         // adjoint of state n+1
  State g0;          // adjoint of state n (may alias g1)
  int ld;
  const int *act_id;
  const float *act;  // [n_act_tot]
  const float *pbar, *mbar, *gv;
  int64_t G;
  double *gact;      // [n_act_tot] accumulated dL/ds
  unsigned *err;
  const float *mat = nullptr;  // per-particle (mu, la, m_p) [3][ld] or null
  float *gmat = nullptr;       // += dL/dmu, dL/dla, dL/dm_p [3][ld] (with mat)
  float *sb_part = nullptr;  // non-null: dL/ds of each particle here (not gact)
  int n = 0;         // substep index (scenes past their horizon are held fixed)
};

// The reverse of substep n's gather fused with the adjoint scatter of
// substep n-1 (3D rollouts): reads state n, the adjoint of state n+1, x and
// F of state n-1 and the adjoint grid of substep n (pbar, mbar, gv); writes
// the adjoint of state n and scatters substep n-1's adjoint into the tile
// boxes (and the overflow grid vbar).
struct AdjFusedArgs {
  const DevScene *scenes;
  CState s;          // state n
  CState g1;         // adjoint of state n+1
  State g0;          // adjoint of state n (must not alias g1)
  CState sp;         // state n-1 (x, F read)
  int ld;
  const int *act_id;
  const float *act;  // [n_act_tot] of substep n
  const float *pbar, *mbar, *gv;  // adjoint grid of substep n
  int64_t G;
  double *gact;      // [n_act_tot] accumulated dL/ds^n (nullable)
  float *vbar;       // overflow adjoint grid of substep n-1
  unsigned *err;
  TileInfo tiles;
  int det = 0;       // deterministic sums (fixed order of a cell's records)
  float *sb_part = nullptr;  // non-null: dL/ds of each particle here (not gact)
  int n = 0;         // substep index (scenes past their horizon are held fixed)
};

struct SortArgs {
  const DevScene *scenes;
  const int *pscene;  // scene of each particle (caller order)
  int N;
  const float *x;
  int ld;
  int tile;           // cells per tile edge
  int *cell_cnt;      // [n_tiles * tile^d], zeroed
  int *tile_cnt;      // [n_tiles], zeroed
  int *ptile, *pcell, *prank;
  unsigned *err;
};

int launch_p2g(int dim, const P2GArgs &a, hipStream_t st);
// One workgroup per tile (n_tiles of them, empty tiles exit at once).
int launch_p2g_tile(int dim, const P2GArgs &a, int n_tiles, hipStream_t st);
int launch_adj_scatter_tile(int dim, const AdjScatterArgs &a, int n_tiles,
                            hipStream_t st);
// Per-cell variants (tiles of 64 cells: 8x8 in 2D, 4x4x4 in 3D): one wave
// per tile, lane = cell, register accumulation over the cell's particles.
// cell_cnt is the binning's per-cell particle count [n_tiles][64].
int launch_p2g_cell(int dim, const P2GArgs &a, const int *cell_cnt,
                    int n_tiles, hipStream_t st);
int launch_adj_scatter_cell(int dim, const AdjScatterArgs &a,
                            const int *cell_cnt, int n_tiles, hipStream_t st);
// Sorted per-cell variants (same tiles): each launch re-sorts a tile's
// particles by their current cell in LDS, so drift does not matter.
// n_blocks: number of tiles in a.tiles.list (or all tiles when it is null).
int launch_p2g_sorted(int dim, const P2GArgs &a, int n_blocks, hipStream_t st);
int launch_adj_scatter_sorted(int dim, const AdjScatterArgs &a, int n_blocks,
                              hipStream_t st);
// Tile edges (cells) with compiled kernels for each dimension.
bool tile_supported(int dim, int B);
int launch_grid(int dim, const GridArgs &a, hipStream_t st);
// Node-tile variants of the grid kernels (binned rollouts with 64-cell
// tiles): every node of node tile t is covered by the boxes of tiles t-1
// and t per axis only, so a wave takes the 64 nodes of one node tile, reads
// the candidates' counts once and skips empty boxes (and node tiles with no
// particle nearby) as a whole.
int launch_grid_nt(int dim, const GridArgs &a, hipStream_t st);
int launch_adj_grid_nt(int dim, const AdjGridArgs &a, hipStream_t st);
int launch_g2p(int dim, const G2PArgs &a, hipStream_t st);
int launch_g2p_p2g_sorted(int dim, const G2P2GArgs &a, int n_blocks, hipStream_t st);
int launch_adj_scatter(int dim, const AdjScatterArgs &a, hipStream_t st);
int launch_adj_grid(int dim, const AdjGridArgs &a, hipStream_t st);
int launch_adj_gather(int dim, const AdjGatherArgs &a, hipStream_t st);
int launch_adj_gather_scatter(int dim, const AdjFusedArgs &a, int n_blocks, hipStream_t st);
// Deterministic mode: per-actuator sums of a substep's per-particle dL/ds
// (tape order) into gact [n_act]; act_scene: scene of each actuator.
int launch_sbar_reduce(const DevScene *scenes, const int *act_scene, int n_act,
                       const int *tile_start, const int *act_id, const float *sb_part,
                       int dim, double *gact, hipStream_t st);
// Deterministic ranks at binning: the particles of each cell listed by
// atomic rank (cell_start: exclusive scan of the cell counts), then each
// cell's list sorted by particle index, which becomes the rank.
int launch_cell_fill(const int *ptile, const int *pcell, const int *prank,
                     const int *cell_start, int cpt, int N, int *list, hipStream_t st);
int launch_cell_sort(const int *cell_start, int n_cells, int *list, int *prank,
                     hipStream_t st);

int launch_mat_field(const DevScene *scenes, const int *pscene, int N,
                     const float *E_p, const float *rho_p, float *mat, hipStream_t st);
int launch_mat_grad(const DevScene *scenes, const int *pscene, int N, const int *perm,
                    const float *gmat, float *g_E, float *g_rho, hipStream_t st);
// The allocation-free single substep's set-up (one scene): descriptors,
// sanitised actuator ids and cleared m, p in the caller's device region.
struct NoAllocArgs {
  DevScene sc;
  int dim, N;
  int64_t nodes, G;     // the scene's nodes; plane stride of gp
  DevScene *scene;
  Chunk *chunks;
  GridBlock *blocks;
  const int *act_id_in;  // caller's ids (device, nullable: all passive)
  int *act_id;           // sanitised copy [N]
  float *gm, *gp;
  unsigned *err;
};
int launch_noalloc_setup(const NoAllocArgs &a, hipStream_t st);
int launch_fill_f32(float *p, int64_t n, hipStream_t st);
int launch_fill_f64(double *p, int64_t n, hipStream_t st);
int launch_fill_i32(int *p, int64_t n, hipStream_t st);

int launch_sort_count(int dim, const SortArgs &a, hipStream_t st);
// Exclusive scan of in[0..n) into out[0..n] (out[n] = total), one workgroup.
int launch_scan_i32(const int *in, int *out, int n, hipStream_t st);
int launch_sort_place(int dim, const SortArgs &a, const int *tile_start,
                      int *perm, hipStream_t st);
int launch_chunk_count(const int *tile_cnt, int n_tiles, int *nch,
                       hipStream_t st);
// flag[i] = tile_cnt[i] > 0; list[pos[i]] = i for flagged tiles.
int launch_nonempty_flag(const int *tile_cnt, int n_tiles, int *flag,
                         hipStream_t st);
// Per node tile of 3D 4^3-cell tiles, the 8 covering tiles holding particles.
int launch_nt_cand(const DevScene *scenes, const int *nt_scene, int n_nt,
                   const int *tile_cnt, int *cand, hipStream_t st);
int launch_compact(const int *flag, const int *pos, int n_tiles, int *list,
                   hipStream_t st);
int launch_build_chunks(const int *tile_cnt, const int *tile_start,
                        const int *chunk_start, const int *tile_scene,
                        int n_tiles, Chunk *chunks, hipStream_t st);
// out = in[perm] (gather) or out[perm] = in (scatter) over every component
// of a state with `ncomp` rows of length N (stride ld).
int launch_permute_rows(const float *in, float *out, const int *perm, int N,
                        int ld, int ncomp, int scatter, hipStream_t st);
int launch_permute_i32(const int *in, int *out, const int *perm, int N,
                       hipStream_t st);
// Closed-loop controller (section IV, Control), one scene: a = tanh(W z + b),
// z = [target, mean x and mean v of each component].  nzs = 2 d n_comp.
struct CtlArgs {
  int dim, N, n_comp, n_act, nz;
  const int *comp;        // component of each particle (binned order), -1 none
  const float *inv_cnt;   // [n_comp] 1 / particles of the component
  const float *x, *v;     // state n ([d][ld])
  int ld;
  float *partial;         // [nzs][rows] per-workgroup sums (entry-major)
  double *sums;           // [nzs]
  unsigned *done;         // workgroups finished (zero between launches)
  const float *W, *b, *target;  // [n_act][nz], [n_act], [d]
  float *act;             // out: [n_act] actuation of this substep
  float *z;               // out: [nz] state vector of this substep (tape)
};
int launch_ctl_forward(const CtlArgs &a, hipStream_t st);
// The reduction and controller evaluation alone, over n_rows partial rows
// written by the previous G2P (launch_g2p with ctl_partial).
int launch_ctl_reduce(const CtlArgs &a, int n_rows, hipStream_t st);
// Rows of partial sums the forward reduction uses for N particles.
int ctl_rows(int N);
struct CtlAdjArgs {
  int dim, N, n_comp, n_act, nz;
  const int *comp;
  const float *inv_cnt;
  const float *W, *act, *z;  // W, a^n and z^n of this substep
  const double *sbar;        // [n_act] dL/ds^n
  double *gW, *gb;           // accumulated [n_act][nz], [n_act]
  float *gx, *gv;            // adjoint of state n ([d][ld]), += broadcast
  int ld;
};
int launch_ctl_adjoint(const CtlAdjArgs &a, hipStream_t st);
int launch_gact_store(const double *src, float *dst, int64_t n, int accumulate,
                      hipStream_t st);
int launch_act_bank_fwd(int T, int n_act, int n_freq, float dt,
                        const float *freq, const float *amp,
                        const float *phase, float *act, hipStream_t st);
int launch_act_bank_bwd(int T, int n_act, int n_freq, float dt,
                        const float *freq, const float *amp,
                        const float *phase, const float *g_act, float *g_amp,
                        float *g_phase, hipStream_t st);

}  // namespace mpm
