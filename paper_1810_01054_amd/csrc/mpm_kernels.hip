// mpm_kernels.hip -- gfx950 kernels of one MLS-MPM substep and its adjoint
// (ChainQueen, arXiv 1810.01054: section III steps 1-3; supplement (A)-(K)).
//
// Work decomposition.  Particles are processed in chunks of CH = 256 (one
// particle per lane, four 64-wide waves).  A chunk's workgroup first reduces
// the bounding box of its particles' stencil bases; when the (box + 2)^d
// grid nodes fit in LDS_NODES, the stencil traffic of the whole chunk goes
// through LDS:
//   * scatters (P2G, adjoint of G2P) accumulate with LDS float atomics and
//     flush the box to HBM with one global atomic per non-empty node;
//   * gathers (G2P, adjoint of P2G) stage the box's node data into LDS with
//     coalesced loads and read the 3^d stencil from there.
// Chunks whose box does not fit take the same path against global memory.
// When particles are binned by tile (rollouts sort them once: tile, then
// rank within its cell, then cell), the 64 lanes of a wave hold 64 distinct
// cells, so the LDS atomics of one instruction never hit the same address.
//
// No MFMA: the work is stencil scatter/gather over streamed particle state,
// not a dense contraction.
#include <float.h>
#include <limits.h>
#include <math.h>

#include <type_traits>

#include "mpm_internal.h"

namespace mpm {

namespace {

// ---------------------------------------------------------------------------
// small dense algebra (row-major d x d, fully unrolled)
// ---------------------------------------------------------------------------

template <int D>
__device__ __forceinline__ float det(const float *A) {
  if constexpr (D == 2) {
    return A[0] * A[3] - A[1] * A[2];
  } else {
    return A[0] * (A[4] * A[8] - A[5] * A[7]) -
           A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
  }
}

// R = A^{-T} = cofactor(A) / J
template <int D>
__device__ __forceinline__ void inv_transpose(const float *A, float J,
                                              float *R) {
  const float iJ = 1.0f / J;
  if constexpr (D == 2) {
    R[0] = A[3] * iJ;
    R[1] = -A[2] * iJ;
    R[2] = -A[1] * iJ;
    R[3] = A[0] * iJ;
  } else {
    R[0] = (A[4] * A[8] - A[5] * A[7]) * iJ;
    R[1] = -(A[3] * A[8] - A[5] * A[6]) * iJ;
    R[2] = (A[3] * A[7] - A[4] * A[6]) * iJ;
    R[3] = -(A[1] * A[8] - A[2] * A[7]) * iJ;
    R[4] = (A[0] * A[8] - A[2] * A[6]) * iJ;
    R[5] = -(A[0] * A[7] - A[1] * A[6]) * iJ;
    R[6] = (A[1] * A[5] - A[2] * A[4]) * iJ;
    R[7] = -(A[0] * A[5] - A[2] * A[3]) * iJ;
    R[8] = (A[0] * A[4] - A[1] * A[3]) * iJ;
  }
}

template <int D>
__device__ __forceinline__ void load_vec(const float *p, int ld, int i,
                                         float *out) {
#pragma unroll
  for (int a = 0; a < D; ++a) out[a] = p[a * ld + i];
}

template <int D>
__device__ __forceinline__ void load_mat(const float *p, int ld, int i,
                                         float *out) {
#pragma unroll
  for (int k = 0; k < D * D; ++k) out[k] = p[k * ld + i];
}

template <int D>
__device__ __forceinline__ void store_vec(float *p, int ld, int i,
                                          const float *v) {
#pragma unroll
  for (int a = 0; a < D; ++a) p[a * ld + i] = v[a];
}

template <int D>
__device__ __forceinline__ void store_mat(float *p, int ld, int i,
                                          const float *v) {
#pragma unroll
  for (int k = 0; k < D * D; ++k) p[k * ld + i] = v[k];
}

__device__ __forceinline__ bool finite_all(const float *v, int n) {
  bool ok = true;
  for (int i = 0; i < n; ++i) ok = ok && isfinite(v[i]);
  return ok;
}

// ---------------------------------------------------------------------------
// quadratic B-spline stencil (Table I: N; base = floor(x/dx - 0.5))
// ---------------------------------------------------------------------------

template <int D>
__device__ __forceinline__ bool stencil_base(const float *xp,
                                             const DevScene &sc, int *base,
                                             float *f, unsigned &eb) {
  bool ok = true;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const float q = xp[a] * sc.inv_dx;
    int b = 0;
    if (!isfinite(q)) {
      eb |= EB_NONFINITE;
      ok = false;
    } else {
      const float qs = q - 0.5f;
      if (qs < -1.0f || qs > (float)sc.n) {
        eb |= EB_DOMAIN;
        ok = false;
      } else {
        b = (int)floorf(qs);
        if (b < 0 || b > sc.n - 3) {
          eb |= EB_DOMAIN;
          ok = false;
        }
      }
    }
    base[a] = b;
    f[a] = q - (float)b;  // in [0.5, 1.5)
  }
  return ok;
}

// Weights w[a][k] of nodes base+k along axis a.
__device__ __forceinline__ void bspline_w(float f, float *w) {
  const float t0 = 1.5f - f, t1 = f - 1.0f, t2 = f - 0.5f;
  w[0] = 0.5f * t0 * t0;
  w[1] = 0.75f - t1 * t1;
  w[2] = 0.5f * t2 * t2;
}

// Derivatives of those weights with respect to the particle coordinate.
__device__ __forceinline__ void bspline_dw(float f, float inv_dx, float *dw) {
  dw[0] = (f - 1.5f) * inv_dx;
  dw[1] = (2.0f - 2.0f * f) * inv_dx;
  dw[2] = (f - 0.5f) * inv_dx;
}

// G2P stencil sums of one 3D particle (section III, G2P), taken axis by axis:
// vn = sum_o N(o) v_o and Bm[a][b] = sum_o N(o) v_o,a (o_b - f_b) with
// N(o) = w[0][o0] w[1][o1] w[2][o2].  Summing along axis 2, then 1, then 0,
// each node velocity enters six multiply-adds (sixteen when every node forms
// N(o) v_o (o - f)^T).  vel(o0, o1, o2, v) fetches the velocity of node
// base + o; the outer axis stays a loop (nine node fetches in flight).  Every
// 3D G2P uses this one summation order, so a state recomputed from the tape
// equals the forward pass's bit for bit.
template <typename Vel>
__device__ __forceinline__ void g2p_sums3(const float (&w)[3][3], const float *f,
                                          Vel &&vel, float *vn, float (&Bm)[3][3]) {
  float wd1[3], wd2[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    wd1[k] = w[1][k] * ((float)k - f[1]);
    wd2[k] = w[2][k] * ((float)k - f[2]);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    vn[a] = 0.0f;
    Bm[a][0] = Bm[a][1] = Bm[a][2] = 0.0f;
  }
#pragma unroll 1
  for (int o0 = 0; o0 < 3; ++o0) {
    float Y0[3] = {}, Y1[3] = {}, Y2[3] = {};
#pragma unroll
    for (int o1 = 0; o1 < 3; ++o1) {
      float Z0[3] = {}, Z2[3] = {};
#pragma unroll
      for (int o2 = 0; o2 < 3; ++o2) {
        float v[3];
        vel(o0, o1, o2, v);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          Z0[a] += w[2][o2] * v[a];
          Z2[a] += wd2[o2] * v[a];
        }
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        Y0[a] += w[1][o1] * Z0[a];
        Y1[a] += wd1[o1] * Z0[a];
        Y2[a] += w[1][o1] * Z2[a];
      }
    }
    const float wx = o0 == 0 ? w[0][0] : (o0 == 1 ? w[0][1] : w[0][2]);
    const float wdx = wx * ((float)o0 - f[0]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      vn[a] += wx * Y0[a];
      Bm[a][0] += wdx * Y0[a];
      Bm[a][1] += wx * Y1[a];
      Bm[a][2] += wx * Y2[a];
    }
  }
}

// ---------------------------------------------------------------------------
// workgroup bounding box of stencil bases
// ---------------------------------------------------------------------------

template <int D>
struct Box {
  int lo[D];
  int e[D];   // node extent per axis (= hi - lo + 3)
  int vol;    // prod e, 0 when the chunk holds no valid particle
  bool lds;   // the box fits in LDS_NODES
};

template <int D>
__device__ __forceinline__ Box<D> chunk_box(bool ok, const int *base) {
  __shared__ int s_red[2 * D][CH / 64];
  int mn[D], mx[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    mn[a] = ok ? base[a] : INT_MAX;
    mx[a] = ok ? base[a] : INT_MIN;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      mn[a] = min(mn[a], __shfl_xor(mn[a], off, 64));
      mx[a] = max(mx[a], __shfl_xor(mx[a], off, 64));
    }
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      s_red[a][wave] = mn[a];
      s_red[D + a][wave] = mx[a];
    }
  }
  __syncthreads();
  Box<D> b;
  int hi[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    int l = s_red[a][0], h = s_red[D + a][0];
#pragma unroll
    for (int w = 1; w < CH / 64; ++w) {
      l = min(l, s_red[a][w]);
      h = max(h, s_red[D + a][w]);
    }
    b.lo[a] = l;
    hi[a] = h;
  }
  if (b.lo[0] > hi[0]) {
    b.vol = 0;
    b.lds = false;
#pragma unroll
    for (int a = 0; a < D; ++a) b.e[a] = 0;
    return b;
  }
  long vol = 1;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    b.e[a] = hi[a] - b.lo[a] + 3;
    vol *= b.e[a];
  }
  b.vol = vol > (long)INT_MAX ? INT_MAX : (int)vol;
  b.lds = vol <= LDS_NODES;
  return b;
}

// LDS slot of the node (base + o) relative to the box.
template <int D>
__device__ __forceinline__ int box_index(const Box<D> &b, const int *base) {
  if constexpr (D == 2) {
    return (base[0] - b.lo[0]) * b.e[1] + (base[1] - b.lo[1]);
  } else {
    return ((base[0] - b.lo[0]) * b.e[1] + (base[1] - b.lo[1])) * b.e[2] +
           (base[2] - b.lo[2]);
  }
}

// Scene-local linear node index of the box slot i.
template <int D>
__device__ __forceinline__ int box_node(const Box<D> &b, int i, int n) {
  if constexpr (D == 2) {
    const int l1 = i % b.e[1], l0 = i / b.e[1];
    return (b.lo[0] + l0) * n + (b.lo[1] + l1);
  } else {
    const int l2 = i % b.e[2];
    const int r = i / b.e[2];
    const int l1 = r % b.e[1], l0 = r / b.e[1];
    return ((b.lo[0] + l0) * n + (b.lo[1] + l1)) * n + (b.lo[2] + l2);
  }
}

template <int D>
__device__ __forceinline__ int node_index(const int *base, int n) {
  if constexpr (D == 2) return base[0] * n + base[1];
  else return (base[0] * n + base[1]) * n + base[2];
}

__device__ __forceinline__ void lds_add(float *p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void gmem_add(float *p, float v) {
  unsafeAtomicAdd(p, v);
}

// ---------------------------------------------------------------------------
// per-particle stress: neo-Hookean P, actuation, G_p (section III, P2G)
// ---------------------------------------------------------------------------

template <int D>
struct Stress {
  float FiT[D * D];
  float Pt[D * D];  // P(F) + F sigma
  float sigma[D];
  float lnJ;
};

// Material of one particle: Lame parameters and mass (the scene's, or the
// per-particle field [3][ld]: mu, la, m_p).
struct Mat {
  float mu, la, mp;
};
__device__ __forceinline__ Mat scene_mat(const DevScene &sc) {
  return Mat{sc.mu, sc.la, sc.mp};
}
__device__ __forceinline__ Mat particle_mat(const float *mat, int ld,
                                            const DevScene &sc, int p) {
  if (mat) return Mat{mat[p], mat[ld + p], mat[2 * ld + p]};
  return scene_mat(sc);
}

// Returns false (and sets eb) when det F <= 0 or is not finite.
template <int D>
__device__ __forceinline__ bool stress(const DevScene &sc, const Mat &m,
                                       const float *F, float s_act,
                                       bool has_act, Stress<D> &S,
                                       unsigned &eb) {
  const float J = det<D>(F);
  if (!isfinite(J)) {
    eb |= EB_NONFINITE;
    return false;
  }
  if (!(J > 0.0f)) {
    eb |= EB_INVERTED;
    return false;
  }
  inv_transpose<D>(F, J, S.FiT);
  S.lnJ = logf(J);
#pragma unroll
  for (int b = 0; b < D; ++b) S.sigma[b] = has_act ? s_act * sc.axis[b] : 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      const int k = a * D + b;
      // P = mu (F - F^-T) + la ln J F^-T;  P_t = P + F sigma
      S.Pt[k] = m.mu * (F[k] - S.FiT[k]) + m.la * S.lnJ * S.FiT[k] +
                F[k] * S.sigma[b];
    }
  return true;
}

// G = kG P_t F^T + m_p C with kG = -(4/dx^2) dt V0.
template <int D>
__device__ __forceinline__ void affine_G(const DevScene &sc, const Mat &m,
                                         const float *Pt, const float *F,
                                         const float *C, float *G) {
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      float s = 0.0f;
#pragma unroll
      for (int g = 0; g < D; ++g) s += Pt[a * D + g] * F[b * D + g];
      G[a * D + b] = sc.kG * s + m.mp * C[a * D + b];
    }
}

// Workgroups go to the eight XCDs round-robin by block index, and each XCD
// has its own L2.  Chunks are in tile order and node blocks in node order,
// so neighbouring work items share grid nodes or tile boxes: give each XCD a
// contiguous run of them (a bijection of the block indices) so that the
// shared data passes through one L2.
__device__ __forceinline__ int xcd_block_id() {
  constexpr int NX = 8;
  const int nb = gridDim.x, b = blockIdx.x;
  const int q = nb / NX, r = nb % NX, x = b % NX, k = b / NX;
  return x * q + min(x, r) + k;
}

// The work items of this workgroup: item xcd_block_id() of a launch with
// one workgroup per item, or (persistent launch with min(n_items, 8) or more
// workgroups, fewer than items) every item of its XCD's contiguous share of
// the items, at a stride of the number of workgroups on that XCD.  No
// barrier may depend on the count.
template <typename F>
__device__ __forceinline__ void for_items(int n_items, bool persistent, F &&f) {
  if (!persistent) {
    f(xcd_block_id());
    return;
  }
  constexpr int NX = 8;
  const int nb = gridDim.x, b = blockIdx.x, x = b % NX, k = b / NX;
  const int nbx = nb / NX + (x < nb % NX ? 1 : 0);
  const int q = n_items / NX, r = n_items % NX;
  const int lo = x * q + min(x, r), hi = lo + q + (x < r ? 1 : 0);
  for (int i = lo + k; i < hi; i += nbx) f(i);
}

// ---------------------------------------------------------------------------
// step 1: P2G scatter
// ---------------------------------------------------------------------------

// Scatter the 3^d stencil of one particle.  Channel values at offset o are
//   val_c = N(o) * (c0[c] + sum_b L[c][b] o_b)   (affine in o),
// plus, when HAS_MASS, channel "mass" N(o) * m0 emitted first.  `sink(o0,
// o1, o2, vals)` receives NCH = D (+1 with mass) values per node.
template <int D, bool HAS_MASS, typename Sink>
__device__ __forceinline__ void scatter_stencil(const float (&w)[D][3],
                                                float m0, const float *c0,
                                                const float (&L)[D][D],
                                                Sink &&sink) {
  constexpr int M = HAS_MASS ? 1 : 0;
  if constexpr (D == 2) {
#pragma unroll
    for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
      for (int o1 = 0; o1 < 3; ++o1) {
        const float N = w[0][o0] * w[1][o1];
        float val[D + M];
        if constexpr (HAS_MASS) val[0] = N * m0;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          float v = c0[a];  // zero offset components left out
          if (o0) v += L[a][0] * o0;
          if (o1) v += L[a][1] * o1;
          val[M + a] = N * v;
        }
        sink(o0, o1, 0, val);
      }
  } else {
#pragma unroll
    for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
      for (int o1 = 0; o1 < 3; ++o1) {
        const float w01 = w[0][o0] * w[1][o1];
#pragma unroll
        for (int o2 = 0; o2 < 3; ++o2) {
          const float N = w01 * w[2][o2];
          float val[D + M];
          if constexpr (HAS_MASS) val[0] = N * m0;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            float v = c0[a];  // zero offset components left out
            if (o0) v += L[a][0] * o0;
            if (o1) v += L[a][1] * o1;
            if (o2) v += L[a][2] * o2;
            val[M + a] = N * v;
          }
          sink(o0, o1, o2, val);
        }
      }
  }
}

// Per-particle P2G quantities (section III, P2G): B-spline weights and the
// affine form of m_p v_p + G_p (x_i - x_p) = c0 + sum_b Gdx[.][b] o_b.
// Returns false (with eb set) for an invalid particle.
template <int D>
__device__ __forceinline__ bool p2g_record(const DevScene &sc, const Mat &m,
                                           const float *F, const float *C,
                                           const float *v, float s_act,
                                           bool has_act, const float *f,
                                           float (&w)[D][3], float *c0,
                                           float (&Gdx)[D][D], unsigned &eb) {
  float G[D * D];
  Stress<D> S;
  if (!stress<D>(sc, m, F, s_act, has_act, S, eb)) return false;
  affine_G<D>(sc, m, S.Pt, F, C, G);
#pragma unroll
  for (int a = 0; a < D; ++a) bspline_w(f[a], w[a]);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float s = m.mp * v[a];
#pragma unroll
    for (int b = 0; b < D; ++b) {
      Gdx[a][b] = G[a * D + b] * sc.dx;
      s -= Gdx[a][b] * f[b];
    }
    c0[a] = s;
  }
  return true;
}

template <int D>
__device__ __forceinline__ bool p2g_particle(const P2GArgs &A,
                                             const DevScene &sc, int p,
                                             const float *xp, const float *f,
                                             float (&w)[D][3], float *c0,
                                             float (&Gdx)[D][D],
                                             unsigned &eb) {
  if (A.n >= sc.t_end) return false;  // past the scene's horizon: held fixed
  float F[D * D], C[D * D], v[D];
  load_mat<D>(A.s.F, A.ld, p, F);
  load_mat<D>(A.s.C, A.ld, p, C);
  load_vec<D>(A.s.v, A.ld, p, v);
  const int j = A.act_id[p];
  const float s_act = j >= 0 ? A.act[sc.act_off + j] : 0.0f;
  return p2g_record<D>(sc, scene_mat(sc), F, C, v, s_act, j >= 0, f, w, c0, Gdx, eb);
}

// The same with the particle's own material (per-particle field when the
// context has one); mpp: its mass, for the scatter's mass channel.
template <int D>
__device__ __forceinline__ bool p2g_particle_m(const P2GArgs &A,
                                               const DevScene &sc, int p,
                                               const float *xp, const float *f,
                                               float (&w)[D][3], float *c0,
                                               float (&Gdx)[D][D], float &mpp,
                                               unsigned &eb) {
  if (A.n >= sc.t_end) return false;  // past the scene's horizon: held fixed
  float F[D * D], C[D * D], v[D];
  load_mat<D>(A.s.F, A.ld, p, F);
  load_mat<D>(A.s.C, A.ld, p, C);
  load_vec<D>(A.s.v, A.ld, p, v);
  const int j = A.act_id[p];
  const float s_act = j >= 0 ? A.act[sc.act_off + j] : 0.0f;
  const Mat m = particle_mat(A.mat, A.ld, sc, p);
  mpp = m.mp;
  return p2g_record<D>(sc, m, F, C, v, s_act, j >= 0, f, w, c0, Gdx, eb);
}

// Per-particle adjoint-scatter quantities (supplement (A)-(C)):
// vt + (4/dx^2) Ct (x_i - x_p) = c0 + sum_b Cdx[.][b] o_b.
// The streams the adjoint scatter reads for particle p: F^n and the adjoint
// of state n+1.
template <int D>
struct AdjScatterIn {
  float F[D * D], gx[D], gv[D], gC[D * D], gF[D * D];
};
template <int D>
__device__ __forceinline__ void adj_scatter_load(const AdjScatterArgs &A, int p,
                                                 AdjScatterIn<D> &in) {
  load_mat<D>(A.s.F, A.ld, p, in.F);
  load_vec<D>(A.g1.x, A.ld, p, in.gx);
  load_vec<D>(A.g1.v, A.ld, p, in.gv);
  load_mat<D>(A.g1.C, A.ld, p, in.gC);
  load_mat<D>(A.g1.F, A.ld, p, in.gF);
}

template <int D>
__device__ __forceinline__ void adj_scatter_particle(const AdjScatterArgs &A,
                                                     const DevScene &sc,
                                                     const AdjScatterIn<D> &in,
                                                     const float *f,
                                                     float (&w)[D][3],
                                                     float *c0,
                                                     float (&Cdx)[D][D]) {
  const float *F = in.F, *gx = in.gx, *gv = in.gv, *gC = in.gC, *gF = in.gF;
  float vt[D], Ct[D * D];
  // (A): dL/dv^{n+1} total = carried + dt dL/dx^{n+1}
#pragma unroll
  for (int a = 0; a < D; ++a) vt[a] = gv[a] + sc.dt * gx[a];
  // (B): dL/dC^{n+1} total = carried + dt dL/dF^{n+1} F^{nT}
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      float s = 0.0f;
#pragma unroll
      for (int g = 0; g < D; ++g) s += gF[a * D + g] * F[b * D + g];
      Ct[a * D + b] = gC[a * D + b] + sc.dt * s;
    }
#pragma unroll
  for (int a = 0; a < D; ++a) bspline_w(f[a], w[a]);
  // (C): vt + (4/dx^2) Ct (x_i - x_p), x_i - x_p = (o - f) dx
  const float cs = sc.Dinv * sc.dx;
  // past the scene's horizon the substep is the identity: nothing to add
  const float on = A.n >= sc.t_end ? 0.0f : 1.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float s = vt[a];
#pragma unroll
    for (int b = 0; b < D; ++b) {
      Cdx[a][b] = on * (cs * Ct[a * D + b]);
      s -= Cdx[a][b] * f[b];
    }
    c0[a] = on * s;
  }
}

// Global-memory sink: one atomic per channel and node.
template <int D, int M>
__device__ __forceinline__ void add_global(float *m, float *p, int64_t G,
                                           int64_t gi, const float *val) {
  if constexpr (M == 1) gmem_add(&m[gi], val[0]);
#pragma unroll
  for (int a = 0; a < D; ++a) gmem_add(&p[a * G + gi], val[M + a]);
}

template <int D>
__device__ __forceinline__ int64_t stencil_gindex(int64_t gbase, int n, int o0,
                                                  int o1, int o2) {
  if constexpr (D == 2) return gbase + o0 * n + o1;
  else return gbase + ((int64_t)o0 * n + o1) * n + o2;
}

// Chunk version (caller-ordered particles): LDS box when the chunk's stencil
// box fits, global atomics otherwise; the LDS box is flushed with one global
// atomic per non-empty node.
template <int D>
__global__ __launch_bounds__(CH) void k_p2g(P2GArgs A) {
  __shared__ float s_grid[(D + 1) * LDS_NODES];
  const Chunk ch = A.chunks[xcd_block_id()];
  const DevScene sc = A.scenes[ch.scene];
  const int t = threadIdx.x;
  const bool active = t < ch.count;
  const int p = ch.start + t;
  unsigned eb = 0;
  float xp[D], f[D];
  int base[D];
  bool ok = false;
  if (active) {
    load_vec<D>(A.s.x, A.ld, p, xp);
    ok = stencil_base<D>(xp, sc, base, f, eb);
  }
  const Box<D> box = chunk_box<D>(ok, base);
  float w[D][3], c0[D], Gdx[D][D], mpp = 0.0f;
  if (ok) ok = p2g_particle_m<D>(A, sc, p, xp, f, w, c0, Gdx, mpp, eb);
  if (box.lds) {
    for (int i = t; i < (D + 1) * LDS_NODES; i += CH) s_grid[i] = 0.0f;
    __syncthreads();
  }
  if (ok) {
    if (box.lds) {
      const int lbase = box_index<D>(box, base);
      scatter_stencil<D, true>(w, mpp, c0, Gdx,
                               [&](int o0, int o1, int o2, const float *val) {
        const int li = D == 2 ? lbase + o0 * box.e[1] + o1
                              : lbase + (o0 * box.e[1] + o1) * box.e[2] + o2;
#pragma unroll
        for (int c = 0; c <= D; ++c) lds_add(&s_grid[c * LDS_NODES + li], val[c]);
      });
    } else {
      const int64_t gbase = sc.g_off + node_index<D>(base, sc.n);
      scatter_stencil<D, true>(w, mpp, c0, Gdx,
                               [&](int o0, int o1, int o2, const float *val) {
        add_global<D, 1>(A.gm, A.gp, A.G,
                         stencil_gindex<D>(gbase, sc.n, o0, o1, o2), val);
      });
    }
  }
  if (eb) atomicOr(A.err, eb);
  if (box.lds) {
    __syncthreads();
    for (int i = t; i < box.vol; i += CH) {
      const float m = s_grid[i];
      if (m != 0.0f) {
        const int64_t gi = sc.g_off + box_node<D>(box, i, sc.n);
        gmem_add(&A.gm[gi], m);
#pragma unroll
        for (int a = 0; a < D; ++a)
          gmem_add(&A.gp[a * A.G + gi], s_grid[(a + 1) * LDS_NODES + i]);
      }
    }
  }
}

// Node origin (scene-local node coordinates) of tile `lt`'s box.
template <int D, int B>
__device__ __forceinline__ void tile_origin(int lt, int nt, int *org) {
#pragma unroll
  for (int a = D - 1; a >= 0; --a) {
    org[a] = (lt % nt) * B - 1;
    lt /= nt;
  }
}

// Position in a stored box plane of box node i (node-major, last axis
// fastest).  A 3D box of a 4^3-cell tile (8^3 nodes) is stored as 2 x 2 x 2
// blocks of 4^3 nodes, each block contiguous: box u spans the node tiles u
// and u+1 of the grid kernels per axis, so the nodes a grid-kernel wave takes
// from one box are one whole block (256 contiguous bytes per channel).
// Other boxes are stored node-major.
template <int D, int B>
__device__ __forceinline__ int box_pos(int i) {
  if constexpr (D == 3 && B == 4) {
    const int l0 = i >> 6, l1 = (i >> 3) & 7, l2 = i & 7;
    const int blk = ((l0 >> 2) * 2 + (l1 >> 2)) * 2 + (l2 >> 2);
    return (blk << 6) | (((l0 & 3) * 4 + (l1 & 3)) * 4 + (l2 & 3));
  } else {
    return i;
  }
}
// The box node stored at position j (inverse of box_pos).
template <int D, int B>
__device__ __forceinline__ int box_node_at(int j) {
  if constexpr (D == 3 && B == 4) {
    const int blk = j >> 6, r = j & 63;
    const int l0 = ((blk >> 2) & 1) * 4 + (r >> 4);
    const int l1 = ((blk >> 1) & 1) * 4 + ((r >> 2) & 3);
    const int l2 = (blk & 1) * 4 + (r & 3);
    return (l0 * 8 + l1) * 8 + l2;
  } else {
    return j;
  }
}

// Tile version (binned particles): one workgroup per tile, LDS accumulation,
// whole box stored with plain coalesced stores; particles whose stencil left
// the box add to the grid with global atomics.
template <int D, int B>
__global__ __launch_bounds__(256) void k_p2g_tile(P2GArgs A) {
  constexpr int S = TileBox<B>::S;
  constexpr int SV = D == 2 ? S * S : S * S * S;
  __shared__ float s_grid[(D + 1) * SV];
  const int tile = blockIdx.x;
  const int cnt = A.tiles.cnt[tile];
  if (cnt == 0) return;
  const DevScene sc = A.scenes[A.tiles.scene[tile]];
  int org[D];
  tile_origin<D, B>(tile - sc.tile_off, sc.nt, org);
  const int t = threadIdx.x;
  for (int i = t; i < (D + 1) * SV; i += 256) s_grid[i] = 0.0f;
  __syncthreads();
  unsigned eb = 0;
  const int start = A.tiles.start[tile];
  for (int j = t; j < cnt; j += 256) {
    const int p = start + j;
    float xp[D], f[D];
    int base[D];
    load_vec<D>(A.s.x, A.ld, p, xp);
    if (!stencil_base<D>(xp, sc, base, f, eb)) continue;
    float w[D][3], c0[D], Gdx[D][D], mpp;
    if (!p2g_particle_m<D>(A, sc, p, xp, f, w, c0, Gdx, mpp, eb)) continue;
    int l[D];
    bool inbox = true;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      l[a] = base[a] - org[a];
      inbox = inbox && l[a] >= 0 && l[a] <= S - 3;
    }
    if (inbox) {
      const int lbase = D == 2 ? l[0] * S + l[1] : (l[0] * S + l[1]) * S + l[2];
      scatter_stencil<D, true>(w, mpp, c0, Gdx,
                               [&](int o0, int o1, int o2, const float *val) {
        const int li = D == 2 ? lbase + o0 * S + o1 : lbase + (o0 * S + o1) * S + o2;
#pragma unroll
        for (int c = 0; c <= D; ++c) lds_add(&s_grid[c * SV + li], val[c]);
      });
    } else {
      const int64_t gbase = sc.g_off + node_index<D>(base, sc.n);
      scatter_stencil<D, true>(w, mpp, c0, Gdx,
                               [&](int o0, int o1, int o2, const float *val) {
        add_global<D, 1>(A.gm, A.gp, A.G,
                         stencil_gindex<D>(gbase, sc.n, o0, o1, o2), val);
      });
    }
  }
  if (eb) atomicOr(A.err, eb);
  __syncthreads();
  float *dst = A.tiles.part + (int64_t)tile * (D + 1) * SV;
  for (int i = t; i < (D + 1) * SV; i += 256)
    dst[i] = s_grid[(i / SV) * SV + box_node_at<D, B>(i % SV)];
}

// ---------------------------------------------------------------------------
// per-cell scatter: one wave per tile of 64 cells, lane = cell
// ---------------------------------------------------------------------------
//
// Binned order is tile, then rank within the cell, then cell, so the r-th
// particles of the 64 cells are contiguous: in round r lane c reads particle
// start + sum_c' min(n_c', r) + #{c' < c : n_c' > r} (a ballot prefix count).
// A lane accumulates the 3^d x NCH contributions of its cell's particles in
// registers (all of them share the cell's stencil base), then adds them into
// its wave's LDS box with plain read-add-write, one stencil offset at a time:
// for a fixed offset the 64 lanes touch 64 distinct nodes, and the LDS
// executes one wave's operations in issue order (the empty asm statements
// keep the compiler from reordering those LDS accesses across offsets).
// Particles that drifted out of their cell add to the box with LDS atomics
// (or to the grid with global atomics when they left the box).

__device__ __forceinline__ int lanes_before(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

#define MPM_LDS_ORDER() asm volatile("" ::: "memory")

// Shared driver.  PART(p, xp, base, f, w, c0, L, eb) -> bool computes one
// particle's affine stencil values; NCH channels, HAS_MASS as in
// scatter_stencil.
template <int D, int NCH, bool HAS_MASS, typename Args, typename Part>
__device__ __forceinline__ void cell_scatter_wave(const Args &A,
                                                  const int *cell_cnt,
                                                  int tile, float *box,
                                                  float *gm, float *gp,
                                                  Part &&part) {
  constexpr int B = D == 2 ? 8 : 4;
  constexpr int S = TileBox<B>::S;
  constexpr int SV = D == 2 ? S * S : S * S * S;
  constexpr int NO = D == 2 ? 9 : 27;
  const int lane = threadIdx.x & 63;
  const DevScene sc = A.scenes[A.tiles.scene[tile]];
  int org[D];
  tile_origin<D, B>(tile - sc.tile_off, sc.nt, org);
  for (int i = lane; i < NCH * SV; i += 64) box[i] = 0.0f;
  MPM_LDS_ORDER();
  int cc[D];
  {
    int l = lane;
#pragma unroll
    for (int a = D - 1; a >= 0; --a) {
      cc[a] = l % B;
      l /= B;
    }
  }
  const int n_l = cell_cnt[tile * 64 + lane];
  const int maxr = wave_max(n_l);
  const int start = A.tiles.start[tile];
  // local box index of this cell's stencil base (cell + 1 cell of slack)
  const int lcell = D == 2 ? (cc[0] + 1) * S + (cc[1] + 1)
                           : ((cc[0] + 1) * S + (cc[1] + 1)) * S + (cc[2] + 1);
  float acc[NO * NCH];
#pragma unroll
  for (int k = 0; k < NO * NCH; ++k) acc[k] = 0.0f;
  unsigned eb = 0;
  int R = 0;
  for (int r = 0; r < maxr; ++r) {
    const bool act = n_l > r;
    const uint64_t mask = __ballot(act);
    if (act) {
      const int p = start + R + lanes_before(mask);
      float xp[D], f[D];
      int base[D];
      load_vec<D>(A.s.x, A.ld, p, xp);
      float w[D][3], c0[D], L[D][D];
      if (stencil_base<D>(xp, sc, base, f, eb) &&
          part(p, xp, base, f, w, c0, L, eb)) {
        bool home = true, inbox = true;
        int l[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
          l[a] = base[a] - org[a];
          home = home && l[a] == cc[a] + 1;
          inbox = inbox && l[a] >= 0 && l[a] <= S - 3;
        }
        if (home) {
          int o = 0;
          scatter_stencil<D, HAS_MASS>(w, sc.mp, c0, L,
                                       [&](int, int, int, const float *val) {
#pragma unroll
            for (int c = 0; c < NCH; ++c) acc[o * NCH + c] += val[c];
            ++o;
          });
        } else if (inbox) {
          const int lb = D == 2 ? l[0] * S + l[1] : (l[0] * S + l[1]) * S + l[2];
          scatter_stencil<D, HAS_MASS>(w, sc.mp, c0, L,
                                       [&](int o0, int o1, int o2, const float *val) {
            const int li = D == 2 ? lb + o0 * S + o1 : lb + (o0 * S + o1) * S + o2;
#pragma unroll
            for (int c = 0; c < NCH; ++c) lds_add(&box[c * SV + li], val[c]);
          });
        } else {
          const int64_t gbase = sc.g_off + node_index<D>(base, sc.n);
          scatter_stencil<D, HAS_MASS>(w, sc.mp, c0, L,
                                       [&](int o0, int o1, int o2, const float *val) {
            add_global<D, HAS_MASS ? 1 : 0>(gm, gp, A.G,
                                            stencil_gindex<D>(gbase, sc.n, o0, o1, o2), val);
          });
        }
      }
    }
    R += __popcll(mask);
  }
  if (eb) atomicOr(A.err, eb);
  MPM_LDS_ORDER();
  // read-add-write, one stencil offset at a time
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    const int o0 = D == 2 ? o / 3 : o / 9;
    const int o1 = D == 2 ? o % 3 : (o / 3) % 3;
    const int o2 = D == 2 ? 0 : o % 3;
    const int li = D == 2 ? lcell + o0 * S + o1 : lcell + (o0 * S + o1) * S + o2;
    float cur[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) cur[c] = box[c * SV + li];
#pragma unroll
    for (int c = 0; c < NCH; ++c) box[c * SV + li] = cur[c] + acc[o * NCH + c];
    MPM_LDS_ORDER();
  }
  float *dst = A.tiles.part + (int64_t)tile * (D + 1) * SV;
  for (int i = lane; i < NCH * SV; i += 64) dst[i] = box[(i / SV) * SV + box_node_at<D, B>(i % SV)];
}

// Sorted per-cell scatter (drift-proof).  One workgroup (4 waves) per tile.
// The tile's particles are processed in batches of 256 PER (PER per thread):
//  1. each thread has PART(p, base, f, w, c0, L, eb) produce its particles'
//     stencil bases and affine stencil records (f, c0, L)
//     and their current cells in the tile box's (B+2)^d cell grid (one cell
//     of drift per side), and takes a rank in each cell (integer LDS atomic);
//  2. an exclusive scan over the cells gives each cell a range; each thread
//     stores its records at their cell's range + rank;
//  3. lane l of every wave takes one cell (the B^d cells of the tile itself
//     first, then the occupied cells of the drift ring), and wave w the
//     stencil offsets q = w, w+4, w+8, ... of all the cell's records.  A lane
//     sums its share in registers (one stencil base per cell), then the
//     waves, one after the other, add their sums into the tile's LDS box with
//     plain read-add-write (for a fixed offset the lanes of a wave touch
//     distinct nodes, and LDS executes a wave's accesses in issue order).
//     LDS float atomics run an order of magnitude slower here; splitting the
//     offsets over the waves keeps the accumulators at a quarter of the
//     stencil and the read-add-write chains short.  Used in 3D.
// At the end the box is stored.  Particles outside the slack ring add to the
// grid with global atomics.  V4 keeps a box node's channels together (one
// 16-byte LDS access per node and offset) instead of one plane per channel.
template <int D>
struct SortedCell {
  static constexpr int B = D == 2 ? 8 : 4;
  static constexpr int S = TileBox<B>::S;
  static constexpr int SV = D == 2 ? S * S : S * S * S;
  static constexpr int BC = B + 2;  // box cells per axis
  static constexpr int NBC = D == 2 ? BC * BC : BC * BC * BC;
  static constexpr int NIN = D == 2 ? B * B : B * B * B;  // the tile's own cells
  static constexpr int REC = D + D + D * D;  // f, c0, L
  static constexpr int NO = D == 2 ? 9 : 27;  // stencil offsets
  static constexpr int WS = 4;                 // offset stride of a wave
  static constexpr int NQ = (NO + WS - 1) / WS;  // offsets per wave (at most)
};

// PM: records carry the particle's mass (per-particle materials).
// DET: deterministic ranks; mask holds, per box cell, one bit per particle
// of the batch (PER * 256 bits).
template <int D, int NCH, int PER, bool V4, bool PM = false, bool DET = false>
struct SortedCellSmem {
  static constexpr int SV = SortedCell<D>::SV;
  static constexpr int MW = PER * 8;  // mask words per cell
  float box[V4 ? 4 * SV : NCH * SV];
  float rec[(SortedCell<D>::REC + (PM ? 1 : 0)) * PER * 256];  // field-major
  short sidx[PER * 256];  // record slot of each sorted position (swizzled positions)
  int cnt[256];
  int off[256];
  short order[256];  // the tile's own cells, then the occupied ring cells
  int wsum[4];
  int nring;
  unsigned mask[DET ? SortedCell<D>::NBC * MW : 1];
};

// Deterministic ranks in a cell (DET scatters): each particle of a batch
// sets its bit (batch index jl) in its cell's mask; the count of a cell is
// its number of set bits and a particle's rank the number of set bits below
// its own, so a cell's records are ordered by batch index whatever order the
// threads ran in.
template <int MW>
__device__ __forceinline__ void det_mark(unsigned *mask, int lc, int jl) {
  atomicOr(&mask[lc * MW + (jl >> 5)], 1u << (jl & 31));
}
template <int MW>
__device__ __forceinline__ int det_count(const unsigned *mask, int c) {
  int n = 0;
#pragma unroll
  for (int w = 0; w < MW; ++w) n += __popc(mask[c * MW + w]);
  return n;
}
template <int MW>
__device__ __forceinline__ int det_rank(const unsigned *mask, int lc, int jl) {
  const unsigned *m = mask + lc * MW;
  int r = 0;
  for (int w = 0; w < (jl >> 5); ++w) r += __popc(m[w]);
  return r + __popc(m[jl >> 5] & ((1u << (jl & 31)) - 1u));
}

// Exclusive scan of cnt[0..256) into off (256 threads).
__device__ __forceinline__ void block_scan_256(const int *cnt, int *off,
                                               int *wsum) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int v = cnt[t];
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  int pre = 0;
  for (int w = 0; w < wave; ++w) pre += wsum[w];
  off[t] = pre + x - v;
}

// Stencil offset q = (o0 * 3 + o1) * 3 + o2 (2D: o0 * 3 + o1).
template <int D, int Q>
struct StencilOffset {
  static constexpr int o0 = D == 2 ? Q / 3 : Q / 9;
  static constexpr int o1 = D == 2 ? Q % 3 : (Q / 3) % 3;
  static constexpr int o2 = D == 2 ? 0 : Q % 3;
};

// One record's contributions at the offsets W, W+WS, ... added into acc.
template <int D, int NCH, bool HAS_MASS, int W, int J = 0>
__device__ __forceinline__ void offsets_add(const float (&w)[D][3], float mp,
                                            const float *c0,
                                            const float (&L)[D][D],
                                            float *acc) {
  constexpr int Q = W + SortedCell<D>::WS * J;
  if constexpr (Q < SortedCell<D>::NO) {
    using O = StencilOffset<D, Q>;
    float N = w[0][O::o0] * w[1][O::o1];
    if constexpr (D == 3) N *= w[2][O::o2];
    int ch = 0;
    if constexpr (HAS_MASS) acc[J * NCH + ch++] += N * mp;
    // terms with a zero offset component are left out (the compiler keeps
    // a multiply by 0.0f, which is not an identity in IEEE arithmetic)
#pragma unroll
    for (int a = 0; a < D; ++a) {
      float v = c0[a];
      if constexpr (O::o0 != 0) v += L[a][0] * (float)O::o0;
      if constexpr (O::o1 != 0) v += L[a][1] * (float)O::o1;
      if constexpr (D == 3 && O::o2 != 0) v += L[a][2] * (float)O::o2;
      acc[J * NCH + ch + a] += N * v;
    }
    offsets_add<D, NCH, HAS_MASS, W, J + 1>(w, mp, c0, L, acc);
  }
}

// LDS bank swizzles of the offset-split scatter.  Records: a cell holds
// about eight of them, so the lanes of a wave (one cell each) read slots
// about 8 apart, which fall on few banks; flipping the low three slot bits
// by bits 6-8 spreads them.  Box nodes (S = 8, 64 nodes per x-plane): the
// 4x4x4 own cells of a wave touch a 4x4 patch in four planes; flipping node
// bits per plane parity moves each plane's patch to other banks (V4: bits 2
// and 3 of the 16-byte node index; planes: bits 2 and 5 of the float index).
__device__ __forceinline__ int rec_slot(int s) { return s ^ ((s >> 6) & 7); }
template <bool V4>
__device__ __forceinline__ int box_slot(int li) {
  const int n0 = li >> 6;
  return V4 ? li ^ (((n0 & 1) << 2) | (((n0 >> 1) & 1) << 3))
            : li ^ (((n0 & 1) << 2) | (((n0 >> 1) & 1) << 5));
}

// The n records of a cell (first slot o; NR slots per field), summed into
// acc at offsets W, W+4, ...
template <int D, int NCH, bool HAS_MASS, int W, bool PM = false>
__device__ __forceinline__ void cell_offsets_sum(const float *rec, int NR,
                                                 const short *sidx, int o, int n,
                                                 float mp, float *acc) {
  for (int k = 0; k < n; ++k) {
    const int ps = sidx ? (int)sidx[rec_slot(o + k)] : rec_slot(o + k);
    float w[D][3], c0[D], L[D][D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      bspline_w(rec[a * NR + ps], w[a]);
      c0[a] = rec[(D + a) * NR + ps];
#pragma unroll
      for (int b = 0; b < D; ++b) L[a][b] = rec[(2 * D + a * D + b) * NR + ps];
    }
    const float mk = PM ? rec[SortedCell<D>::REC * NR + ps] : mp;
    offsets_add<D, NCH, HAS_MASS, W>(w, mk, c0, L, acc);
  }
}

// Read-add-write of acc (offsets W, W+WS, ...) into the box around lcell.
template <int D, int NCH, bool V4, int W, int J = 0>
__device__ __forceinline__ void offsets_flush(float *box, int lcell,
                                              const float *acc) {
  constexpr int Q = W + SortedCell<D>::WS * J;
  if constexpr (Q < SortedCell<D>::NO) {
    using O = StencilOffset<D, Q>;
    constexpr int S = SortedCell<D>::S, SV = SortedCell<D>::SV;
    const int li = box_slot<V4>(D == 2 ? lcell + O::o0 * S + O::o1
                                       : lcell + (O::o0 * S + O::o1) * S + O::o2);
    if constexpr (V4) {
      float4 *node = reinterpret_cast<float4 *>(box) + li;
      float4 cur = *node;
      cur.x += acc[J * NCH + 0];
      cur.y += acc[J * NCH + 1];
      if constexpr (NCH > 2) cur.z += acc[J * NCH + 2];
      if constexpr (NCH > 3) cur.w += acc[J * NCH + 3];
      *node = cur;
    } else {
      float cur[NCH];
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) cur[ch] = box[ch * SV + li];
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) box[ch * SV + li] = cur[ch] + acc[J * NCH + ch];
    }
    MPM_LDS_ORDER();
    offsets_flush<D, NCH, V4, W, J + 1>(box, lcell, acc);
  }
}

// PM: the part callback also returns the particle's mass, which the
// records carry (per-particle materials); otherwise the scene's mass.
// With a `cell(p, base, eb)` callback (split mode) the ranks come first from
// the particles' stencil bases alone, and part() runs after the cell scan
// and writes each record straight to its sorted slot, so no record is held
// in registers across the batch (part() is then called for every particle
// of the tile, also when it has no record).
// Node tiles reached by a particle that adds to the grid with global atomics
// (stencil base `base`, nodes base .. base+2 per axis): flagged so that the
// node-tile grid kernels also visit them.
template <int D>
__device__ __forceinline__ void mark_dirty(const TileInfo &T, const DevScene &sc,
                                           const int *base) {
  if (T.n_over) {
    // one atomic per wave: the lowest calling lane adds the wave's count
    const unsigned long long m = __ballot(1);
    if ((threadIdx.x & 63) == __ffsll((long long)m) - 1) atomicAdd(T.n_over, __popcll(m));
  }
  if (!T.nt_dirty) return;
  int lo[D], hi[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    lo[a] = (base[a] + 1) / T.B;
    hi[a] = (base[a] + 3) / T.B;
  }
#pragma unroll
  for (int k = 0; k < (1 << D); ++k) {
    int idx = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) idx = idx * sc.nnt + (((k >> (D - 1 - a)) & 1) ? hi[a] : lo[a]);
    T.nt_dirty[sc.nt_off + idx] = 1;
  }
}

struct NoCell {};
template <int D, int NCH, bool HAS_MASS, int PER, bool V4, bool PM = false,
          bool DET = false, typename Args, typename Part, typename Cell = NoCell>
__device__ __forceinline__ void sorted_cell_scatter(
    const Args &A, int tile, SortedCellSmem<D, NCH, PER, V4, PM, DET> &sm, float *gm,
    float *gp, Part &&part, Cell &&cell = Cell{}) {
  constexpr int MW = SortedCellSmem<D, NCH, PER, V4, PM, DET>::MW;
  constexpr bool SPLIT = !std::is_same<std::decay_t<Cell>, NoCell>::value;
  using SC = SortedCell<D>;
  constexpr int S = SC::S, SV = SC::SV, BC = SC::BC, NBC = SC::NBC,
                NIN = SC::NIN, REC = SC::REC, B = SC::B, NQ = SC::NQ;
  constexpr int RECP = REC + (PM ? 1 : 0);
  constexpr int BOXF = V4 ? 4 * SV : NCH * SV;  // floats in the box
  constexpr int NR = PER * 256;                 // record slots per field
  static_assert(!V4 || NCH <= 4, "V4 holds at most four channels");
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const DevScene sc = A.scenes[A.tiles.scene[tile]];
  int org[D];
  tile_origin<D, B>(tile - sc.tile_off, sc.nt, org);
  const int cnt = A.tiles.cnt[tile];
  const int start = A.tiles.start[tile];
  for (int i = t; i < BOXF; i += 256) sm.box[i] = 0.0f;
  sm.cnt[t] = 0;
  if constexpr (DET)
    for (int i = t; i < NBC * MW; i += 256) sm.mask[i] = 0u;
  // is box cell t one of the tile's own cells (1..B on every axis)?
  bool own = t < NBC;
  {
    int l = t;
#pragma unroll
    for (int a = D - 1; a >= 0; --a) {
      const int c = l % BC;
      own = own && c >= 1 && c <= B;
      l /= BC;
    }
  }
  {
    // the own cells take the first NIN slots of the order, in cell order
    const unsigned long long bal = __ballot(own);
    if (lane == 0) sm.wsum[wave] = __popcll(bal);
    __syncthreads();
    int before = __popcll(bal & ((1ull << lane) - 1));
    for (int w = 0; w < wave; ++w) before += sm.wsum[w];
    if (own) sm.order[before] = (short)t;
  }
  unsigned eb = 0;
  __syncthreads();
  // non-split: each record goes to LDS slot h * 256 + t as soon as it is
  // built (no record stays in registers across the batch) and the sorted
  // order is an index of those slots
  const short *sidx = SPLIT ? nullptr : sm.sidx;
  for (int b0 = 0; b0 < cnt; b0 += PER * 256) {
    // 1. records, cells and ranks of up to PER particles per thread
    int lc[PER], rank[PER];
    if constexpr (SPLIT) {
#pragma unroll
      for (int h = 0; h < PER; ++h) {
        lc[h] = -1;
        rank[h] = 0;
        const int j = b0 + h * 256 + t;
        int base[D];
        if (j < cnt && cell(start + j, base, eb)) {
          int l[D];
          bool inbox = true;
#pragma unroll
          for (int a = 0; a < D; ++a) {
            l[a] = base[a] - org[a];
            inbox = inbox && l[a] >= 0 && l[a] < BC;
          }
          if (inbox) {
            lc[h] = D == 2 ? l[0] * BC + l[1] : (l[0] * BC + l[1]) * BC + l[2];
            if constexpr (DET) det_mark<MW>(sm.mask, lc[h], h * 256 + t);
            else rank[h] = atomicAdd(&sm.cnt[lc[h]], 1);
          }
        }
      }
    }
#pragma unroll
    for (int h = 0; h < (SPLIT ? 0 : PER); ++h) {
      lc[h] = -1;
      rank[h] = 0;
      const int j = b0 + h * 256 + t;
      const int p = start + j;
      float f[D], w[D][3], c0[D], L[D][D], mpp = sc.mp;
      int base[D];
      bool got = false;
      if (j < cnt) {
        if constexpr (PM) got = part(p, base, f, w, c0, L, mpp, eb);
        else got = part(p, base, f, w, c0, L, eb);
      }
      if (!got) continue;
      int l[D];
      bool inbox = true;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        l[a] = base[a] - org[a];
        inbox = inbox && l[a] >= 0 && l[a] < BC;
      }
      if (inbox) {
        lc[h] = D == 2 ? l[0] * BC + l[1] : (l[0] * BC + l[1]) * BC + l[2];
        const int us = h * 256 + t;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          sm.rec[a * NR + us] = f[a];
          sm.rec[(D + a) * NR + us] = c0[a];
#pragma unroll
          for (int b = 0; b < D; ++b) sm.rec[(2 * D + a * D + b) * NR + us] = L[a][b];
        }
        if constexpr (PM) sm.rec[REC * NR + us] = mpp;
        if constexpr (DET) det_mark<MW>(sm.mask, lc[h], h * 256 + t);
        else rank[h] = atomicAdd(&sm.cnt[lc[h]], 1);
      } else {
        const int64_t gbase = sc.g_off + node_index<D>(base, sc.n);
        scatter_stencil<D, HAS_MASS>(w, mpp, c0, L,
                                     [&](int o0, int o1, int o2, const float *val) {
          add_global<D, HAS_MASS ? 1 : 0>(gm, gp, A.G,
                                          stencil_gindex<D>(gbase, sc.n, o0, o1, o2), val);
        });
        mark_dirty<D>(A.tiles, sc, base);
      }
    }
    __syncthreads();
    if constexpr (DET) {
      if (t < NBC) sm.cnt[t] = det_count<MW>(sm.mask, t);
#pragma unroll
      for (int h = 0; h < PER; ++h)
        if (lc[h] >= 0) rank[h] = det_rank<MW>(sm.mask, lc[h], h * 256 + t);
      __syncthreads();
    }
    // 2. cell ranges; records to their sorted slots; the occupied ring
    //    cells (particles that drifted out of the tile) after the own cells
    block_scan_256(sm.cnt, sm.off, sm.wsum);
    __syncthreads();
    {
      const bool ring = t < NBC && !own && sm.cnt[t] > 0;
      const unsigned long long bal = __ballot(ring);
      if (lane == 0) sm.wsum[wave] = __popcll(bal);
      __syncthreads();
      int before = __popcll(bal & ((1ull << lane) - 1));
      for (int w = 0; w < wave; ++w) before += sm.wsum[w];
      if (ring) sm.order[NIN + before] = (short)t;
      if (t == 0) sm.nring = sm.wsum[0] + sm.wsum[1] + sm.wsum[2] + sm.wsum[3];
    }
    if constexpr (SPLIT) {
      // records after the scan: each goes straight to its sorted slot, or
      // to the grid when its particle is outside the box's slack
#pragma unroll 1
      for (int h = 0; h < PER; ++h) {
        const int j = b0 + h * 256 + t;
        if (j >= cnt) continue;
        int base[D];
        float f[D], w[D][3], c0[D], L[D][D], mpp = sc.mp;
        bool got;
        if constexpr (PM) got = part(start + j, base, f, w, c0, L, mpp, eb);
        else got = part(start + j, base, f, w, c0, L, eb);
        if (!got) continue;
        if (lc[h] >= 0) {
          const int ps = rec_slot(sm.off[lc[h]] + rank[h]);
#pragma unroll
          for (int a = 0; a < D; ++a) {
            sm.rec[a * NR + ps] = f[a];
            sm.rec[(D + a) * NR + ps] = c0[a];
#pragma unroll
            for (int b = 0; b < D; ++b) sm.rec[(2 * D + a * D + b) * NR + ps] = L[a][b];
          }
          if constexpr (PM) sm.rec[REC * NR + ps] = mpp;
        } else {
          const int64_t gbase = sc.g_off + node_index<D>(base, sc.n);
          scatter_stencil<D, HAS_MASS>(w, mpp, c0, L,
                                       [&](int o0, int o1, int o2, const float *val) {
            add_global<D, HAS_MASS ? 1 : 0>(gm, gp, A.G,
                                            stencil_gindex<D>(gbase, sc.n, o0, o1, o2), val);
          });
          mark_dirty<D>(A.tiles, sc, base);
        }
      }
    } else {
#pragma unroll
      for (int h = 0; h < PER; ++h)
        if (lc[h] >= 0) sm.sidx[rec_slot(sm.off[lc[h]] + rank[h])] = (short)(h * 256 + t);
    }
    __syncthreads();
    // 3. per-cell sums of this wave's offsets, then the waves' read-add-write
    //    into the box, one wave at a time
    const int nslot = NIN + sm.nring;
    for (int ps = 0; ps * 64 < nslot; ++ps) {
      const int slot = ps * 64 + lane;
      const int c = slot < nslot ? sm.order[slot] : 0;
      const int n = slot < nslot ? sm.cnt[c] : 0;
      const int o = sm.off[c];
      float acc[NQ * NCH];
#pragma unroll
      for (int k = 0; k < NQ * NCH; ++k) acc[k] = 0.0f;
      switch (wave) {
        case 0: cell_offsets_sum<D, NCH, HAS_MASS, 0, PM>(sm.rec, NR, sidx, o, n, sc.mp, acc); break;
        case 1: cell_offsets_sum<D, NCH, HAS_MASS, 1, PM>(sm.rec, NR, sidx, o, n, sc.mp, acc); break;
        case 2: cell_offsets_sum<D, NCH, HAS_MASS, 2, PM>(sm.rec, NR, sidx, o, n, sc.mp, acc); break;
        default: cell_offsets_sum<D, NCH, HAS_MASS, 3, PM>(sm.rec, NR, sidx, o, n, sc.mp, acc); break;
      }
      int cc[D];
      {
        int l = c;
#pragma unroll
        for (int a = D - 1; a >= 0; --a) {
          cc[a] = l % BC;
          l /= BC;
        }
      }
      const int lcell = D == 2 ? cc[0] * S + cc[1] : (cc[0] * S + cc[1]) * S + cc[2];
      for (int fw = 0; fw < 4; ++fw) {
        if (wave == fw && n > 0) {
          MPM_LDS_ORDER();
          switch (fw) {
            case 0: offsets_flush<D, NCH, V4, 0>(sm.box, lcell, acc); break;
            case 1: offsets_flush<D, NCH, V4, 1>(sm.box, lcell, acc); break;
            case 2: offsets_flush<D, NCH, V4, 2>(sm.box, lcell, acc); break;
            default: offsets_flush<D, NCH, V4, 3>(sm.box, lcell, acc); break;
          }
        }
        __syncthreads();
      }
    }
    sm.cnt[t] = 0;
    if constexpr (DET)
      for (int i = t; i < NBC * MW; i += 256) sm.mask[i] = 0u;
    __syncthreads();
  }
  if (eb) atomicOr(A.err, eb);
  // 4. store the tile box (one plane per channel)
  float *dst = A.tiles.part + (int64_t)tile * (D + 1) * SV;
  if constexpr (V4) {
    for (int i = t; i < SV; i += 256) {
      const float4 a =
          reinterpret_cast<const float4 *>(sm.box)[box_slot<true>(box_node_at<D, B>(i))];
      dst[i] = a.x;
      dst[SV + i] = a.y;
      if constexpr (NCH > 2) dst[2 * SV + i] = a.z;
      if constexpr (NCH > 3) dst[3 * SV + i] = a.w;
    }
  } else {
    for (int i = t; i < NCH * SV; i += 256)
      dst[i] = sm.box[(i / SV) * SV + box_slot<false>(box_node_at<D, B>(i % SV))];
  }
}

// 2D variant of the sorted scatter (tiles of 8 x 8 cells, about four
// particles per cell): records are sorted as above, then thread c takes box
// cell c and sums all its records at all nine offsets (the 100 box cells
// keep two waves busy), and each wave adds its lanes' sums into its own LDS
// box (read-add-write, the four chains run in parallel); the four boxes are
// summed at the end.  On the 64-scene 2D batch this beats the offset split.
template <int D, int NCH, bool PM = false, bool DET = false>
struct WaveBoxSmem {
  static constexpr int MW = 16;  // mask words per cell (batches of 512)
  float box[4][NCH * SortedCell<D>::SV];
  float rec[512 * (SortedCell<D>::REC + (PM ? 1 : 0))];
  int cnt[256];
  int off[256];
  int wsum[4];
  unsigned mask[DET ? SortedCell<D>::NBC * MW : 1];
};

template <int D, int NCH, bool HAS_MASS, bool PM = false, bool DET = false,
          typename Args, typename Part>
__device__ __forceinline__ void sorted_cell_scatter_wb(const Args &A, int tile,
                                                       WaveBoxSmem<D, NCH, PM, DET> &sm,
                                                    float *gm, float *gp,
                                                    Part &&part) {
  using SC = SortedCell<D>;
  constexpr int S = SC::S, SV = SC::SV, BC = SC::BC, NBC = SC::NBC,
                B = SC::B;
  constexpr int REC = SC::REC + (PM ? 1 : 0);  // record floats (PM: + mass)
  constexpr int NO = D == 2 ? 9 : 27;
  constexpr int PER = 2;  // particles prepared per thread and batch
  const int t = threadIdx.x, wave = t >> 6;
  const DevScene sc = A.scenes[A.tiles.scene[tile]];
  int org[D];
  tile_origin<D, B>(tile - sc.tile_off, sc.nt, org);
  const int cnt = A.tiles.cnt[tile];
  const int start = A.tiles.start[tile];
  constexpr int MW = WaveBoxSmem<D, NCH, PM, DET>::MW;
  float *mybox = sm.box[wave];
  for (int i = t & 63; i < NCH * SV; i += 64) mybox[i] = 0.0f;
  sm.cnt[t] = 0;
  if constexpr (DET)
    for (int i = t; i < NBC * MW; i += 256) sm.mask[i] = 0u;
  int cc[D];  // this thread's box cell in phase 3 (t < NBC)
  {
    int l = t;
#pragma unroll
    for (int a = D - 1; a >= 0; --a) {
      cc[a] = l % BC;
      l /= BC;
    }
  }
  float acc[NO * NCH];
#pragma unroll
  for (int k = 0; k < NO * NCH; ++k) acc[k] = 0.0f;
  unsigned eb = 0;
  __syncthreads();
  for (int b0 = 0; b0 < cnt; b0 += PER * 256) {
    // 1. records, cells and ranks of up to 512 particles
    int lc[PER], rank[PER];
    float rec[PER][REC];
#pragma unroll
    for (int h = 0; h < PER; ++h) {
      lc[h] = -1;
      rank[h] = 0;
      const int j = b0 + h * 256 + t;
      if (j >= cnt) continue;
      const int p = start + j;
      float xp[D], f[D], w[D][3], c0[D], L[D][D], mpp = sc.mp;
      int base[D];
      load_vec<D>(A.s.x, A.ld, p, xp);
      if (!stencil_base<D>(xp, sc, base, f, eb)) continue;
      bool got;
      if constexpr (PM) got = part(p, xp, f, w, c0, L, mpp, eb);
      else got = part(p, xp, f, w, c0, L, eb);
      if (!got) continue;
      int l[D];
      bool inbox = true;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        l[a] = base[a] - org[a];
        inbox = inbox && l[a] >= 0 && l[a] < BC;
      }
      if (inbox) {
        lc[h] = D == 2 ? l[0] * BC + l[1] : (l[0] * BC + l[1]) * BC + l[2];
#pragma unroll
        for (int a = 0; a < D; ++a) {
          rec[h][a] = f[a];
          rec[h][D + a] = c0[a];
#pragma unroll
          for (int b = 0; b < D; ++b) rec[h][2 * D + a * D + b] = L[a][b];
        }
        if constexpr (PM) rec[h][REC - 1] = mpp;
        if constexpr (DET) det_mark<MW>(sm.mask, lc[h], h * 256 + t);
        else rank[h] = atomicAdd(&sm.cnt[lc[h]], 1);
      } else {
        const int64_t gbase = sc.g_off + node_index<D>(base, sc.n);
        scatter_stencil<D, HAS_MASS>(w, mpp, c0, L,
                                     [&](int o0, int o1, int o2, const float *val) {
          add_global<D, HAS_MASS ? 1 : 0>(gm, gp, A.G,
                                          stencil_gindex<D>(gbase, sc.n, o0, o1, o2), val);
        });
        mark_dirty<D>(A.tiles, sc, base);
      }
    }
    __syncthreads();
    if constexpr (DET) {
      if (t < NBC) sm.cnt[t] = det_count<MW>(sm.mask, t);
#pragma unroll
      for (int h = 0; h < PER; ++h)
        if (lc[h] >= 0) rank[h] = det_rank<MW>(sm.mask, lc[h], h * 256 + t);
      __syncthreads();
    }
    // 2. cell ranges; records to their sorted slots
    block_scan_256(sm.cnt, sm.off, sm.wsum);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < PER; ++h) {
      if (lc[h] < 0) continue;
      float *dst = sm.rec + (sm.off[lc[h]] + rank[h]) * REC;
#pragma unroll
      for (int k = 0; k < REC; ++k) dst[k] = rec[h][k];
    }
    __syncthreads();
    // 3. per-cell accumulation in registers
    if (t < NBC) {
      const int n = sm.cnt[t], o = sm.off[t];
      for (int k = 0; k < n; ++k) {
        const float *r = sm.rec + (o + k) * REC;
        float w[D][3], c0[D], L[D][D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
          bspline_w(r[a], w[a]);
          c0[a] = r[D + a];
#pragma unroll
          for (int b = 0; b < D; ++b) L[a][b] = r[2 * D + a * D + b];
        }
        int oi = 0;
        scatter_stencil<D, HAS_MASS>(w, PM ? r[REC - 1] : sc.mp, c0, L,
                                     [&](int, int, int, const float *val) {
#pragma unroll
          for (int c = 0; c < NCH; ++c) acc[oi * NCH + c] += val[c];
          ++oi;
        });
      }
    }
    __syncthreads();
    sm.cnt[t] = 0;
    if constexpr (DET)
      for (int i = t; i < NBC * MW; i += 256) sm.mask[i] = 0u;
    __syncthreads();
  }
  if (eb) atomicOr(A.err, eb);
  // 4. per-wave read-add-write of the accumulators into the wave's box
  if (t < NBC) {
    const int lcell = D == 2 ? cc[0] * S + cc[1] : (cc[0] * S + cc[1]) * S + cc[2];
    MPM_LDS_ORDER();
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      const int o0 = D == 2 ? o / 3 : o / 9;
      const int o1 = D == 2 ? o % 3 : (o / 3) % 3;
      const int o2 = D == 2 ? 0 : o % 3;
      const int li = D == 2 ? lcell + o0 * S + o1 : lcell + (o0 * S + o1) * S + o2;
      float cur[NCH];
#pragma unroll
      for (int c = 0; c < NCH; ++c) cur[c] = mybox[c * SV + li];
#pragma unroll
      for (int c = 0; c < NCH; ++c) mybox[c * SV + li] = cur[c] + acc[o * NCH + c];
      MPM_LDS_ORDER();
    }
  }
  __syncthreads();
  // 5. sum the four wave boxes, store the tile box
  float *dst = A.tiles.part + (int64_t)tile * (D + 1) * SV;
  for (int i = t; i < NCH * SV; i += 256)
    dst[i] = (sm.box[0][i] + sm.box[1][i]) + (sm.box[2][i] + sm.box[3][i]);
}


// 3D: both scatters take batches of 512 (a full tile in one pass: one sort
// and one set of read-add-write chains per tile); P2G keeps its four
// channels node-major, the adjoint scatter's three channels are planes.
// 2D: the per-wave-box variant above.
template <int D, bool DET>
__global__ __launch_bounds__(256) void k_p2g_sorted(P2GArgs A) {
  const int tile = A.tiles.list ? A.tiles.list[blockIdx.x] : blockIdx.x;
  if (A.tiles.cnt[tile] == 0) return;
  const DevScene sc = A.scenes[A.tiles.scene[tile]];
  if constexpr (D == 2) {
    __shared__ WaveBoxSmem<D, D + 1, false, DET> sm;
    sorted_cell_scatter_wb<D, D + 1, true>(
        A, tile, sm, A.gm, A.gp,
        [&](int p, const float *xp, const float *f, float (&w)[D][3],
            float *c0, float (&L)[D][D], unsigned &eb) {
          return p2g_particle<D>(A, sc, p, xp, f, w, c0, L, eb);
        });
  } else {
    __shared__ SortedCellSmem<D, D + 1, 2, true, false, DET> sm;
    sorted_cell_scatter<D, D + 1, true, 2, true>(
        A, tile, sm, A.gm, A.gp,
        [&](int p, int *base, float *f, float (&w)[D][3], float *c0,
            float (&L)[D][D], unsigned &eb) {
          float xp[D];
          load_vec<D>(A.s.x, A.ld, p, xp);
          return stencil_base<D>(xp, sc, base, f, eb) &&
                 p2g_particle<D>(A, sc, p, xp, f, w, c0, L, eb);
        });
  }
}

// The same with per-particle materials: each record also carries the
// particle's mass.
template <int D, bool DET>
__global__ __launch_bounds__(256) void k_p2g_sorted_pm(P2GArgs A) {
  const int tile = A.tiles.list ? A.tiles.list[blockIdx.x] : blockIdx.x;
  if (A.tiles.cnt[tile] == 0) return;
  const DevScene sc = A.scenes[A.tiles.scene[tile]];
  if constexpr (D == 2) {
    __shared__ WaveBoxSmem<D, D + 1, true, DET> sm;
    sorted_cell_scatter_wb<D, D + 1, true, true>(
        A, tile, sm, A.gm, A.gp,
        [&](int p, const float *xp, const float *f, float (&w)[D][3],
            float *c0, float (&L)[D][D], float &mpp, unsigned &eb) {
          return p2g_particle_m<D>(A, sc, p, xp, f, w, c0, L, mpp, eb);
        });
  } else {
    __shared__ SortedCellSmem<D, D + 1, 2, true, true, DET> sm;
    sorted_cell_scatter<D, D + 1, true, 2, true, true>(
        A, tile, sm, A.gm, A.gp,
        [&](int p, int *base, float *f, float (&w)[D][3], float *c0,
            float (&L)[D][D], float &mpp, unsigned &eb) {
          float xp[D];
          load_vec<D>(A.s.x, A.ld, p, xp);
          return stencil_base<D>(xp, sc, base, f, eb) &&
                 p2g_particle_m<D>(A, sc, p, xp, f, w, c0, L, mpp, eb);
        });
  }
}

template <int D, bool DET>
__global__ __launch_bounds__(256) void k_adj_scatter_sorted(AdjScatterArgs A) {
  const int tile = A.tiles.list ? A.tiles.list[blockIdx.x] : blockIdx.x;
  if (A.tiles.cnt[tile] == 0) return;
  const DevScene sc = A.scenes[A.tiles.scene[tile]];
  if constexpr (D == 2) {
    __shared__ WaveBoxSmem<D, D, false, DET> sm;
    sorted_cell_scatter_wb<D, D, false>(
        A, tile, sm, nullptr, A.vbar,
        [&](int p, const float *, const float *f, float (&w)[D][3], float *c0,
            float (&L)[D][D], unsigned &) {
          AdjScatterIn<D> in;
          adj_scatter_load<D>(A, p, in);
          adj_scatter_particle<D>(A, sc, in, f, w, c0, L);
          return true;
        });
  } else {
    __shared__ SortedCellSmem<D, D, 2, false, false, DET> sm;
    sorted_cell_scatter<D, D, false, 2, false>(
        A, tile, sm, nullptr, A.vbar,
        [&](int p, int *base, float *f, float (&w)[D][3], float *c0,
            float (&L)[D][D], unsigned &eb) {
          // all of the particle's streams requested at once (one HBM
          // round trip instead of two)
          float xp[D];
          AdjScatterIn<D> in;
          load_vec<D>(A.s.x, A.ld, p, xp);
          adj_scatter_load<D>(A, p, in);
          if (!stencil_base<D>(xp, sc, base, f, eb)) return false;
          adj_scatter_particle<D>(A, sc, in, f, w, c0, L);
          return true;
        });
  }
}

// G2P of substep n and the sorted P2G of substep n+1 in one pass over a
// tile (3D): the tile's box of grid velocities is staged in LDS, each thread
// gathers its particles (section III, G2P), writes state n+1 (x and F only,
// unless the tape keeps state n+1), and hands the new state straight to the
// scatter's record step (section III, P2G), so state n+1 is not read back
// from HBM.  Particles whose stencil left the box
// gather from HBM.
// PM: per-particle materials (the records carry each particle's mass).
template <int D, bool PM, bool DET>
__global__ __launch_bounds__(256, 3) void k_g2p_p2g_sorted(G2P2GArgs A) {
  static_assert(D == 3, "the fused pass is built for 3D tiles");
  using SC = SortedCell<D>;
  constexpr int S = SC::S, SV = SC::SV, BC = SC::BC, B = SC::B;
  __shared__ SortedCellSmem<D, D + 1, 2, true, PM, DET> sm;
  __shared__ float4 s_v[SV];  // node-major grid velocities of the tile box
  const int tile = A.tiles.list ? A.tiles.list[blockIdx.x] : blockIdx.x;
  if (A.tiles.cnt[tile] == 0) return;
  const DevScene sc = A.scenes[A.tiles.scene[tile]];
  int org[D];
  tile_origin<D, B>(tile - sc.tile_off, sc.nt, org);
  for (int i = threadIdx.x; i < SV; i += 256) {
    const int g[3] = {org[0] + i / (S * S), org[1] + (i / S) % S, org[2] + i % S};
    const bool in = g[0] >= 0 && g[0] < sc.n && g[1] >= 0 && g[1] < sc.n &&
                    g[2] >= 0 && g[2] < sc.n;
    const int64_t gi = sc.g_off + ((int64_t)g[0] * sc.n + g[1]) * sc.n + g[2];
    s_v[i] = in ? make_float4(A.gv[gi], A.gv[A.G + gi], A.gv[2 * A.G + gi], 0.0f)
                : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
  // (the scatter synchronises before its record step reads s_v)
  // past the scene's horizon (substep n >= t_end) state n is carried over
  // unchanged; state n+1 is kept whole once the horizon is reached
  const bool frozen = A.n >= sc.t_end;
  const bool write_vc = A.write_vc || A.n + 1 >= sc.t_end;
  auto part = [&](int p, int *base, float *f, float (&w)[D][3], float *c0,
                  float (&L)[D][D], float &mpp, unsigned &eb) {
        float x[D], f0[D], F[D * D];
        int b0[D];
        if (frozen) {
          float a[D * D];
          load_vec<D>(A.s.x, A.ld, p, a);
          store_vec<D>(A.out.x, A.ld, p, a);
          load_vec<D>(A.s.v, A.ld, p, a);
          store_vec<D>(A.out.v, A.ld, p, a);
          load_mat<D>(A.s.C, A.ld, p, a);
          store_mat<D>(A.out.C, A.ld, p, a);
          load_mat<D>(A.s.F, A.ld, p, a);
          store_mat<D>(A.out.F, A.ld, p, a);
          return false;
        }
        load_vec<D>(A.s.x, A.ld, p, x);
        load_mat<D>(A.s.F, A.ld, p, F);
        if (!stencil_base<D>(x, sc, b0, f0, eb)) {
          // keep state n+1 defined (the rollout reports the error)
          float z[D * D] = {};
          store_vec<D>(A.out.x, A.ld, p, x);
          store_vec<D>(A.out.v, A.ld, p, z);
          store_mat<D>(A.out.C, A.ld, p, z);
          store_mat<D>(A.out.F, A.ld, p, F);
          return false;
        }
        int lb[D];
        bool inb = true;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          lb[a] = b0[a] - org[a];
          inb = inb && lb[a] >= 0 && lb[a] < BC;
        }
        const int lbase = (lb[0] * S + lb[1]) * S + lb[2];
        const int64_t gbase = sc.g_off + node_index<D>(b0, sc.n);
        float w0[D][3];
#pragma unroll
        for (int a = 0; a < D; ++a) bspline_w(f0[a], w0[a]);
        float vn[D], Bm[D][D];  // sum N v_i, sum N v_i (o - f)^T
        // every lane of the wave inside the box (the common case): LDS only
        if (__all(inb)) {
          g2p_sums3(w0, f0, [&](int o0, int o1, int o2, float *v) {
            const float4 n4 = s_v[lbase + (o0 * S + o1) * S + o2];
            v[0] = n4.x;
            v[1] = n4.y;
            v[2] = n4.z;
          }, vn, Bm);
        } else {
          g2p_sums3(w0, f0, [&](int o0, int o1, int o2, float *v) {
            if (inb) {
              const float4 n4 = s_v[lbase + (o0 * S + o1) * S + o2];
              v[0] = n4.x;
              v[1] = n4.y;
              v[2] = n4.z;
            } else {
              const int64_t gi = gbase + ((int64_t)o0 * sc.n + o1) * sc.n + o2;
#pragma unroll
              for (int a = 0; a < D; ++a) v[a] = A.gv[a * A.G + gi];
            }
          }, vn, Bm);
        }
        // C' = (4/dx^2) sum N v_i (x_i - x_p)^T; F' = (I + dt C') F;
        // x' = x + dt v'
        const float cs = sc.Dinv * sc.dx;
        float Cn[D * D], Fn[D * D], xn[D];
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int b = 0; b < D; ++b) Cn[a * D + b] = cs * Bm[a][b];
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int b = 0; b < D; ++b) {
            float acc = F[a * D + b];
#pragma unroll
            for (int g = 0; g < D; ++g) acc += sc.dt * Cn[a * D + g] * F[g * D + b];
            Fn[a * D + b] = acc;
          }
#pragma unroll
        for (int a = 0; a < D; ++a) xn[a] = x[a] + sc.dt * vn[a];
        if (!(finite_all(xn, D) && finite_all(vn, D) && finite_all(Cn, D * D) &&
              finite_all(Fn, D * D)))
          eb |= EB_NONFINITE;
        // the next substep's G2P reads only x and F; v and C are written
        // where the tape keeps state n+1
        store_vec<D>(A.out.x, A.ld, p, xn);
        store_mat<D>(A.out.F, A.ld, p, Fn);
        if (write_vc) {
          store_vec<D>(A.out.v, A.ld, p, vn);
          store_mat<D>(A.out.C, A.ld, p, Cn);
        }
        // the record of state n+1 for the scatter (none past the horizon)
        if (A.n + 1 >= sc.t_end) return false;
        if (!stencil_base<D>(xn, sc, base, f, eb)) return false;
        const int j = A.act_id[p];
        const float s_act = j >= 0 ? A.act[sc.act_off + j] : 0.0f;
        const Mat m = PM ? particle_mat(A.mat, A.ld, sc, p) : scene_mat(sc);
        mpp = m.mp;
        return p2g_record<D>(sc, m, Fn, Cn, vn, s_act, j >= 0, f, w, c0, L, eb);
      };
  if constexpr (PM) {
    sorted_cell_scatter<D, D + 1, true, 2, true, true>(A, tile, sm, A.gm, A.gp, part);
  } else {
    sorted_cell_scatter<D, D + 1, true, 2, true>(
        A, tile, sm, A.gm, A.gp,
        [&](int p, int *base, float *f, float (&w)[D][3], float *c0,
            float (&L)[D][D], unsigned &eb) {
          float mpp;
          return part(p, base, f, w, c0, L, mpp, eb);
        });
  }
}

template <int D>
__global__ __launch_bounds__(256) void k_p2g_cell(P2GArgs A, const int *cell_cnt,
                                                  int n_tiles) {
  constexpr int B = D == 2 ? 8 : 4;
  constexpr int S = TileBox<B>::S;
  constexpr int SV = D == 2 ? S * S : S * S * S;
  __shared__ float s_box[4][(D + 1) * SV];
  const int wave = threadIdx.x >> 6;
  const int tile = blockIdx.x * 4 + wave;
  if (tile >= n_tiles || A.tiles.cnt[tile] == 0) return;  // per wave
  cell_scatter_wave<D, D + 1, true>(
      A, cell_cnt, tile, s_box[wave], A.gm, A.gp,
      [&](int p, const float *xp, const int *, const float *f, float (&w)[D][3],
          float *c0, float (&L)[D][D], unsigned &eb) {
        const DevScene sc = A.scenes[A.tiles.scene[tile]];
        return p2g_particle<D>(A, sc, p, xp, f, w, c0, L, eb);
      });
}

template <int D>
__global__ __launch_bounds__(256) void k_adj_scatter_cell(AdjScatterArgs A,
                                                          const int *cell_cnt,
                                                          int n_tiles) {
  constexpr int B = D == 2 ? 8 : 4;
  constexpr int S = TileBox<B>::S;
  constexpr int SV = D == 2 ? S * S : S * S * S;
  __shared__ float s_box[4][D * SV];
  const int wave = threadIdx.x >> 6;
  const int tile = blockIdx.x * 4 + wave;
  if (tile >= n_tiles || A.tiles.cnt[tile] == 0) return;  // per wave
  cell_scatter_wave<D, D, false>(
      A, cell_cnt, tile, s_box[wave], nullptr, A.vbar,
      [&](int p, const float *, const int *, const float *f, float (&w)[D][3],
          float *c0, float (&L)[D][D], unsigned &) {
        const DevScene sc = A.scenes[A.tiles.scene[tile]];
        AdjScatterIn<D> in;
        adj_scatter_load<D>(A, p, in);
        adj_scatter_particle<D>(A, sc, in, f, w, c0, L);
        return true;
      });
}

// Sum over the tile boxes covering scene-local node `li` (coordinates g) of
// channels [c_lo, c_lo + NC) into acc.  Tile t's box spans nodes
// [t B - 1, t B + B + 2], so at most two tiles per axis cover a node (B >= 4):
// the 2^D candidates are enumerated with fixed trip counts, all tile counts
// are loaded at once and then all box entries (two dependent memory round
// trips per node instead of two per covering tile); the adds keep the order
// of the candidates (axis 0 slowest), the order of the nested tile loops.
template <int D, int B, int NC>
__device__ __forceinline__ bool add_tile_boxes(const DevScene &sc, int li,
                                               const int *tile_cnt,
                                               const float *part, int nch,
                                               int c_lo, float *acc) {
  static_assert(B >= 4, "two tiles per axis cover a node only for B >= 4");
  constexpr int S = TileBox<B>::S;
  constexpr int SV = D == 2 ? S * S : S * S * S;
  constexpr int K = 1 << D;
  int g[D], tlo[D], thi[D];
  int r = li;
#pragma unroll
  for (int a = D - 1; a >= 0; --a) {
    g[a] = r % sc.n;
    r /= sc.n;
  }
#pragma unroll
  for (int a = 0; a < D; ++a) {
    thi[a] = min((g[a] + 1) / B, sc.nt - 1);
    tlo[a] = g[a] >= 3 ? (g[a] - 3) / B : 0;
  }
  int tile[K], loc[K], cnt[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    // a candidate past thi on some axis is clamped to a covering tile, so
    // its count load is in bounds and none waits behind a branch; its count
    // is then dropped
    bool ok = true;
    int t_lin = 0, l = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int t = min(tlo[a] + ((k >> (D - 1 - a)) & 1), thi[a]);
      ok = ok && tlo[a] + ((k >> (D - 1 - a)) & 1) <= thi[a];
      t_lin = t_lin * sc.nt + t;
      l = l * S + (g[a] - (t * B - 1));
    }
    tile[k] = sc.tile_off + t_lin;
    loc[k] = l;
    const int c = tile_cnt[tile[k]];
    cnt[k] = ok ? c : 0;
  }
  float val[K][NC];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    // an empty candidate reads the first box's entries instead (one cached
    // line for the whole wave, value dropped below): no branch, and no HBM
    // traffic for boxes that no kernel wrote
    const float *bx =
        part + (cnt[k] != 0 ? ((int64_t)tile[k] * nch + c_lo) * SV + box_pos<D, B>(loc[k]) : 0);
#pragma unroll
    for (int c = 0; c < NC; ++c) val[k][c] = bx[c * SV];
  }
  bool covered = false;
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (cnt[k] != 0) {
      covered = true;
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] += val[k][c];
    }
  return covered;
}

// Returns whether any non-empty tile's box covers the node.
template <int D, int NC>
__device__ __forceinline__ bool add_tile_boxes_any(int B, const DevScene &sc,
                                                   int li, const int *tile_cnt,
                                                   const float *part, int nch,
                                                   int c_lo, float *acc) {
  if constexpr (D == 2) {
    if (B == 8) return add_tile_boxes<2, 8, NC>(sc, li, tile_cnt, part, nch, c_lo, acc);
    return add_tile_boxes<2, 16, NC>(sc, li, tile_cnt, part, nch, c_lo, acc);
  } else {
    if (B == 4) return add_tile_boxes<3, 4, NC>(sc, li, tile_cnt, part, nch, c_lo, acc);
    return add_tile_boxes<3, 8, NC>(sc, li, tile_cnt, part, nch, c_lo, acc);
  }
}

// ---------------------------------------------------------------------------
// step 2: grid operations (v = p/m, gravity, sticky walls)
// ---------------------------------------------------------------------------

template <int D>
__device__ __forceinline__ bool is_wall(int li, int n, int wall) {
  bool w = false;
#pragma unroll
  for (int a = D - 1; a >= 0; --a) {
    const int ia = li % n;
    li /= n;
    w = w || ia < wall || ia >= n - wall;
  }
  return w;
}

// Friction projection (supplement, friction projection gradients (L)) of a
// node velocity against the face with inward normal s e_a (s = +-1), in
// place: l_n = s v_a, v_t = v without its a component, l_t =
// sqrt(|v_t|^2 + eps), l*_t = max(l_t + c min(l_n, 0), 0),
// v* = l*_t v_t / l_t + max(l_n, 0) s e_a.
constexpr float FRICTION_EPS = 1e-12f;

template <int D>
__device__ __forceinline__ void friction_face(float *v, int a, float s, float c) {
  const float ln = s * v[a];
  float lt2 = 0.0f;
#pragma unroll
  for (int b = 0; b < D; ++b)
    if (b != a) lt2 += v[b] * v[b];
  const float lt = sqrtf(lt2 + FRICTION_EPS);
  const float lts = fmaxf(lt + c * fminf(ln, 0.0f), 0.0f);
#pragma unroll
  for (int b = 0; b < D; ++b)
    v[b] = b == a ? fmaxf(ln, 0.0f) * s : lts * (v[b] / lt);
}

// Reverse of friction_face at input velocity v: vb = dL/dv* in, dL/dv out.
// H(x) = [x >= 0], R = l_t + c min(l_n, 0); the normal component of the
// reverse collapses to s (c H(R) H(-l_n) dL/dl*_t + H(l_n) s vb_a) because
// v_t has no a component.
template <int D>
__device__ __forceinline__ void friction_face_bwd(const float *v, int a, float s,
                                                  float c, float *vb) {
  const float ln = s * v[a];
  float lt2 = 0.0f;
#pragma unroll
  for (int b = 0; b < D; ++b)
    if (b != a) lt2 += v[b] * v[b];
  const float lt = sqrtf(lt2 + FRICTION_EPS);
  const float R = lt + c * fminf(ln, 0.0f);
  const float lts = fmaxf(R, 0.0f);
  const float HR = R >= 0.0f ? 1.0f : 0.0f;
  float ltsb = 0.0f, sdot = 0.0f;
#pragma unroll
  for (int b = 0; b < D; ++b)
    if (b != a) {
      ltsb += vb[b] * (v[b] / lt);   // dL/dl*_t
      sdot += v[b] * (vb[b] * lts);  // v_t . dL/dv^_t
    }
  const float ltb = -sdot / (lt * lt) + ltsb * HR;
  const float na = s * (ltsb * HR * c * (-ln >= 0.0f ? 1.0f : 0.0f) +
                        (ln >= 0.0f ? 1.0f : 0.0f) * s * vb[a]);
#pragma unroll
  for (int b = 0; b < D; ++b)
    vb[b] = b == a ? na : (ltb * v[b] + vb[b] * lts) / lt;
}

template <int D>
__device__ __forceinline__ void node_coords(int li, int n, int *idx) {
#pragma unroll
  for (int a = D - 1; a >= 0; --a) {
    idx[a] = li % n;
    li /= n;
  }
}

// Boundary condition on a wall node, in place (bc = 1: one projection per
// face whose band holds the node, axis order, low face first).
template <int D>
__device__ __forceinline__ void wall_bc(const DevScene &sc, int li, float *v) {
  if (sc.bc == 0) {
#pragma unroll
    for (int a = 0; a < D; ++a) v[a] = 0.0f;
    return;
  }
  int idx[D];
  node_coords<D>(li, sc.n, idx);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    if (idx[a] < sc.wall) friction_face<D>(v, a, 1.0f, sc.fric);
    if (idx[a] >= sc.n - sc.wall) friction_face<D>(v, a, -1.0f, sc.fric);
  }
}

// Reverse of wall_bc: v = velocity before the condition (overwritten with
// the velocity after it), vb = dL/dv after -> dL/dv before.
template <int D>
__device__ __forceinline__ void wall_bc_bwd(const DevScene &sc, int li, float *v,
                                            float *vb) {
  if (sc.bc == 0) {
#pragma unroll
    for (int a = 0; a < D; ++a) v[a] = vb[a] = 0.0f;
    return;
  }
  int idx[D];
  node_coords<D>(li, sc.n, idx);
  // inputs of the (at most 2 D) face stages
  float vin[2 * D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const bool on = h == 0 ? idx[a] < sc.wall : idx[a] >= sc.n - sc.wall;
      if (on) {
#pragma unroll
        for (int b = 0; b < D; ++b) vin[2 * a + h][b] = v[b];
        friction_face<D>(v, a, h == 0 ? 1.0f : -1.0f, sc.fric);
      }
    }
#pragma unroll
  for (int a = D - 1; a >= 0; --a)
#pragma unroll
    for (int h = 1; h >= 0; --h) {
      const bool on = h == 0 ? idx[a] < sc.wall : idx[a] >= sc.n - sc.wall;
      if (on) friction_face_bwd<D>(vin[2 * a + h], a, h == 0 ? 1.0f : -1.0f, sc.fric, vb);
    }
}

// Grid operations at one node (section III step 2 with gravity and the wall
// condition): v = p/m + dt g where m > 0, else 0; then wall_bc on wall
// nodes.
template <int D>
__device__ __forceinline__ void node_velocity(const DevScene &sc, int li,
                                              float m, const float *p,
                                              float *v) {
  const bool wall = is_wall<D>(li, sc.n, sc.wall);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    // explicit roundings (no contraction into an FMA): the grid kernel and
    // the G2P that rebuilds velocities from stored (m, p) get the same bits
    float va = 0.0f;
    if (m > 0.0f) va = __fadd_rn(p[a] / m, __fmul_rn(sc.dt, sc.g[a]));
    v[a] = va;
  }
  if (wall) wall_bc<D>(sc, li, v);
}

template <int D>
__global__ __launch_bounds__(256) void k_grid(GridArgs A) {
  const GridBlock gb = A.blocks[xcd_block_id()];
  if ((int)threadIdx.x >= gb.count) return;
  const DevScene sc = A.scenes[gb.scene];
  const int li = gb.start + threadIdx.x;
  const int64_t gi = sc.g_off + li;
  float mp[D + 1];  // m, p (direct adds + tile boxes)
  mp[0] = A.gm[gi];
#pragma unroll
  for (int a = 0; a < D; ++a) mp[1 + a] = A.gp[a * A.G + gi];
  const bool direct = mp[0] != 0.0f;
  if (A.part) {
    const bool covered =
        add_tile_boxes_any<D, D + 1>(A.B, sc, li, A.tile_cnt, A.part, D + 1, 0, mp);
    // a node that no particle reached keeps m = p = 0 and is never read with
    // a non-zero weight: skip it (its buffers hold finite earlier values)
    if (!covered && !direct) return;
  }
  float v[D];
  node_velocity<D>(sc, li, mp[0], mp + 1, v);
#pragma unroll
  for (int a = 0; a < D; ++a) A.gv[a * A.G + gi] = v[a];
  if (A.zero_mp && direct) {
    A.gm[gi] = 0.0f;
#pragma unroll
    for (int a = 0; a < D; ++a) A.gp[a * A.G + gi] = 0.0f;
  }
  if (A.out_m) {
    A.out_m[gi] = mp[0];
#pragma unroll
    for (int a = 0; a < D; ++a) A.out_p[a * A.G + gi] = mp[1 + a];
  }
}

// A node tile of a binned scene (64-cell tiles: B = 4 in 3D, 8 in 2D): node
// tile t holds nodes tB-1 .. tB+B-2 per axis, lane (l0, l1[, l2]) the node
// t B - 1 + l, and the boxes of tiles t-1 and t per axis are the only ones
// that can cover its nodes (box u spans nodes uB-1 .. uB+B+2: the tile's
// cells, the 2-node stencil reach and one cell of slack per side).  Box t
// covers the whole node tile; box t-1 reaches only nodes up to tB+2, which
// is all of them for B = 4 but half of them for B = 8.
template <int D, int B>
struct NodeTile {
  static constexpr int K = 1 << D;
  int li;          // scene-local node index of this lane
  bool valid;      // the node lies in the grid
  int tile[K];     // global tile of candidate k (axis 0 slowest)
  int loc[K];      // this node's index in candidate k's box
  bool nz[K];      // candidate k exists and holds particles (uniform)
  bool cov[K];     // candidate k's box covers this lane's node
  bool any;
};

template <int D, int B>
__device__ __forceinline__ NodeTile<D, B> node_tile(const DevScene &sc, int lt,
                                                    const int *tile_cnt) {
  constexpr int S = TileBox<B>::S;
  NodeTile<D, B> r;
  int t[D], g[D];
  {
    int l = lt, ll = (int)threadIdx.x;
#pragma unroll
    for (int a = D - 1; a >= 0; --a) {
      t[a] = l % sc.nnt;
      l /= sc.nnt;
      g[a] = t[a] * B - 1 + ll % B;
      ll /= B;
    }
  }
  r.valid = true;
  r.li = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    r.valid = r.valid && g[a] >= 0 && g[a] < sc.n;
    r.li = r.li * sc.n + g[a];
  }
  r.any = false;
#pragma unroll
  for (int k = 0; k < NodeTile<D, B>::K; ++k) {
    bool ok = true, cov = true;
    int tl = 0, lc = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int u = t[a] - 1 + ((k >> (D - 1 - a)) & 1);
      const int l = g[a] - (u * B - 1);
      ok = ok && u >= 0 && u < sc.nt;
      cov = cov && l >= 0 && l < S;
      tl = tl * sc.nt + (u >= 0 && u < sc.nt ? u : 0);
      lc = lc * S + l;
    }
    r.tile[k] = sc.tile_off + tl;
    r.loc[k] = lc;
    r.nz[k] = ok && tile_cnt[r.tile[k]] != 0;
    r.cov[k] = cov;
    r.any = r.any || r.nz[k];
  }
  return r;
}

// Candidate table of the 3D node-tile kernels, built once per binning: for
// node tile ntg the global index of each of its 8 covering tiles (tiles t-1
// and t per axis, axis 0 slowest) that exists and holds particles, else -1.
// With 4^3-cell tiles every candidate's box covers the whole node tile, as
// its block (1 - offset) per axis (box_pos), so the grid kernels read the
// boxes from this table without waiting for the tile counts.
__global__ __launch_bounds__(256) void k_nt_cand(const DevScene *scenes,
                                                 const int *nt_scene, int n_nt,
                                                 const int *tile_cnt, int *cand) {
  const int ntg = blockIdx.x * 256 + threadIdx.x;
  if (ntg >= n_nt) return;
  const DevScene sc = scenes[nt_scene[ntg]];
  int t[3], l = ntg - sc.nt_off;
#pragma unroll
  for (int a = 2; a >= 0; --a) {
    t[a] = l % sc.nnt;
    l /= sc.nnt;
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    bool ok = true;
    int tl = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int u = t[a] - 1 + ((k >> (2 - a)) & 1);
      ok = ok && u >= 0 && u < sc.nt;
      tl = tl * sc.nt + (ok ? u : 0);
    }
    const int tile = sc.tile_off + tl;
    cand[(int64_t)ntg * 8 + k] = ok && tile_cnt[tile] != 0 ? tile : -1;
  }
}

// Box entries of node tile ntg's lane from its candidate table (3D, 4^3-cell
// tiles): NC channels of each candidate (zeros for none).
template <int NC>
__device__ __forceinline__ bool nt_cand_boxes(const int *nt_cand, const float *part,
                                              int ntg, float (&val)[8][NC]) {
  constexpr int SV = 512;
  const int lane = threadIdx.x & 63;
  bool any = false;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int tk = nt_cand[(int64_t)ntg * 8 + k];
    any = any || tk >= 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) val[k][c] = 0.0f;
    if (tk >= 0) {
      const int blk = ((1 - ((k >> 2) & 1)) * 2 + (1 - ((k >> 1) & 1))) * 2 + (1 - (k & 1));
      const float *bx = part + (int64_t)tk * 4 * SV + blk * 64 + lane;
#pragma unroll
      for (int c = 0; c < NC; ++c) val[k][c] = bx[c * SV];
    }
  }
  return any;
}

// Node index (scene-local) of this lane in node tile ntg and whether it lies
// in the grid (3D, 4^3-node node tiles).
__device__ __forceinline__ bool nt_node(const DevScene &sc, int ntg, int *li) {
  int l = ntg - sc.nt_off, ll = (int)threadIdx.x & 63, g[3];
#pragma unroll
  for (int a = 2; a >= 0; --a) {
    g[a] = (l % sc.nnt) * 4 - 1 + ll % 4;
    l /= sc.nnt;
    ll /= 4;
  }
  *li = (g[0] * sc.n + g[1]) * sc.n + g[2];
  return g[0] >= 0 && g[0] < sc.n && g[1] >= 0 && g[1] < sc.n && g[2] >= 0 && g[2] < sc.n;
}

// Grid operations over node tiles (see k_grid): direct adds (only where a
// particle beyond its box's slack flagged the node tile) then the candidate
// boxes in the nested-loop order.
template <int D>
__device__ __forceinline__ void grid_nt_item(const GridArgs &A, int ntg) {
  if constexpr (D == 3) {
    if (A.nt_cand) {
      // the box loads go out with the scene and flag loads (candidate table)
      float val[8][4];
      const bool any = nt_cand_boxes<4>(A.nt_cand, A.part, ntg, val);
      const bool dirty = A.nt_dirty[ntg] != 0;
      if (!any && !dirty) return;
      const DevScene sc = A.scenes[A.nt_scene[ntg]];
      int li;
      if (!nt_node(sc, ntg, &li)) return;
      const int64_t gi = sc.g_off + li;
      float mp[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      if (dirty) {
        mp[0] = A.gm[gi];
#pragma unroll
        for (int a = 0; a < 3; ++a) mp[1 + a] = A.gp[a * A.G + gi];
      }
      const bool direct = mp[0] != 0.0f;
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int c = 0; c < 4; ++c) mp[c] += val[k][c];
      float v[3];
      node_velocity<3>(sc, li, mp[0], mp + 1, v);
#pragma unroll
      for (int a = 0; a < 3; ++a) A.gv[a * A.G + gi] = v[a];
      if (A.zero_mp && direct) {
        A.gm[gi] = 0.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a) A.gp[a * A.G + gi] = 0.0f;
      }
      if (A.out_m) {
        A.out_m[gi] = mp[0];
#pragma unroll
        for (int a = 0; a < 3; ++a) A.out_p[a * A.G + gi] = mp[1 + a];
      }
      return;
    }
  }
  constexpr int B = D == 2 ? 8 : 4;
  constexpr int S = TileBox<B>::S, SV = D == 2 ? S * S : S * S * S;
  const DevScene sc = A.scenes[A.nt_scene[ntg]];
  const NodeTile<D, B> nt = node_tile<D, B>(sc, ntg - sc.nt_off, A.tile_cnt);
  const bool dirty = A.nt_dirty[ntg] != 0;
  if ((!nt.any && !dirty) || !nt.valid) return;
  const int64_t gi = sc.g_off + nt.li;
  float mp[D + 1];
#pragma unroll
  for (int c = 0; c <= D; ++c) mp[c] = 0.0f;
  if (dirty) {
    mp[0] = A.gm[gi];
#pragma unroll
    for (int a = 0; a < D; ++a) mp[1 + a] = A.gp[a * A.G + gi];
  }
  const bool direct = mp[0] != 0.0f;
  float val[NodeTile<D, B>::K][D + 1];
#pragma unroll
  for (int k = 0; k < NodeTile<D, B>::K; ++k)
    if (nt.nz[k] && nt.cov[k]) {
      const float *bx = A.part + (int64_t)nt.tile[k] * (D + 1) * SV + box_pos<D, B>(nt.loc[k]);
#pragma unroll
      for (int c = 0; c <= D; ++c) val[k][c] = bx[c * SV];
    }
#pragma unroll
  for (int k = 0; k < NodeTile<D, B>::K; ++k)
    if (nt.nz[k] && nt.cov[k]) {
#pragma unroll
      for (int c = 0; c <= D; ++c) mp[c] += val[k][c];
    }
  float v[D];
  node_velocity<D>(sc, nt.li, mp[0], mp + 1, v);
#pragma unroll
  for (int a = 0; a < D; ++a) A.gv[a * A.G + gi] = v[a];
  if (A.zero_mp && direct) {
    A.gm[gi] = 0.0f;
#pragma unroll
    for (int a = 0; a < D; ++a) A.gp[a * A.G + gi] = 0.0f;
  }
  if (A.out_m) {
    A.out_m[gi] = mp[0];
#pragma unroll
    for (int a = 0; a < D; ++a) A.out_p[a * A.G + gi] = mp[1 + a];
  }
}

// P: persistent launch (a few workgroups per CU loop over the node tiles).
template <int D, bool P>
__global__ __launch_bounds__(64) void k_grid_nt(GridArgs A) {
  for_items(A.n_nt, P, [&](int ntg) { grid_nt_item<D>(A, ntg); });
}

// ---------------------------------------------------------------------------
// step 3: G2P gather + F/C/x update
// ---------------------------------------------------------------------------

// Closed-loop controller sums (section IV, Control): 2 d n_comp <= 96
// entries (x_a of component c at 2 d c + a, v_a at 2 d c + d + a).
constexpr int CTL_MAX_NZS = 96;

// Adds this wave's particles to its LDS row of component sums: the lanes of
// one component at a time are reduced with a reduce-scatter butterfly (the
// 2d values padded to 8: 10 cross-lane steps), lane group v ending with the
// total of value v.  c < 0: the lane contributes nothing.  Every lane of the
// wave must call it.
template <int D>
__device__ __forceinline__ void ctl_wave_add(int c, const float *val8, float *row) {
  const int lane = threadIdx.x & 63;
  const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8;
  const int vi = (h5 ? 4 : 0) + (h4 ? 2 : 0) + (h3 ? 1 : 0);
  unsigned long long todo = __ballot(c >= 0);
  while (todo) {
    const int src = __ffsll((long long)todo) - 1;
    const int cc = __shfl(c, src, 64);
    const bool mine = c == cc;
    float q[4], u[2];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float lo = mine ? val8[k] : 0.0f, hi = mine ? val8[k + 4] : 0.0f;
      q[k] = (h5 ? hi : lo) + __shfl_xor(h5 ? lo : hi, 32, 64);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k)
      u[k] = (h4 ? q[k + 2] : q[k]) + __shfl_xor(h4 ? q[k] : q[k + 2], 16, 64);
    float w = (h3 ? u[1] : u[0]) + __shfl_xor(h3 ? u[0] : u[1], 8, 64);
    w += __shfl_xor(w, 4, 64);
    w += __shfl_xor(w, 2, 64);
    w += __shfl_xor(w, 1, 64);
    if ((lane & 7) == 0 && vi < 2 * D) row[2 * D * cc + vi] += w;
    todo &= ~__ballot(mine);
  }
}

// CTL: also the controller's per-workgroup component sums of the new state
// (row = chunk of the partial array, entry-major), so the controller of the
// next substep only reduces the rows.
template <int D, bool CTL>
__global__ __launch_bounds__(CH) void k_g2p(G2PArgs A) {
  // staged node velocities: planes in 2D, node-major float4 in 3D
  __shared__ float s_v[D == 3 ? 4 * LDS_NODES : D * LDS_NODES];
  __shared__ float s_ctl[CTL ? 4 : 1][CTL ? CTL_MAX_NZS : 1];
  const int chunk = xcd_block_id();
  const Chunk ch = A.chunks[chunk];
  const DevScene sc = A.scenes[ch.scene];
  const int t = threadIdx.x;
  const bool active = t < ch.count;
  const int p = ch.start + t;
  if (A.n >= sc.t_end) {
    // past the scene's horizon: the state is carried over unchanged
    if (active) {
      float a[D * D];
      load_vec<D>(A.s.x, A.ld, p, a);
      store_vec<D>(A.out.x, A.ld, p, a);
      load_vec<D>(A.s.v, A.ld, p, a);
      store_vec<D>(A.out.v, A.ld, p, a);
      load_mat<D>(A.s.C, A.ld, p, a);
      store_mat<D>(A.out.C, A.ld, p, a);
      load_mat<D>(A.s.F, A.ld, p, a);
      store_mat<D>(A.out.F, A.ld, p, a);
    }
    return;
  }
  if constexpr (CTL)
    for (int i = t & 63; i < CTL_MAX_NZS; i += 64) s_ctl[t >> 6][i] = 0.0f;
  unsigned eb = 0;
  float xp[D], f[D];
  int base[D];
  bool ok = false;
  if (active) {
    load_vec<D>(A.s.x, A.ld, p, xp);
    ok = stencil_base<D>(xp, sc, base, f, eb);
  }
  const Box<D> box = chunk_box<D>(ok, base);
  // grid velocity at scene-local node li (from v, or from stored m and p)
  auto vel = [&](int li, float *v) {
    const int64_t gi = sc.g_off + li;
    if (A.gm) {
      float pp[D];
#pragma unroll
      for (int a = 0; a < D; ++a) pp[a] = A.gp[a * A.G + gi];
      node_velocity<D>(sc, li, A.gm[gi], pp, v);
    } else {
#pragma unroll
      for (int a = 0; a < D; ++a) v[a] = A.gv[a * A.G + gi];
    }
  };
  if (box.lds) {
    for (int i = t; i < box.vol; i += CH) {
      float v[D];
      vel(box_node<D>(box, i, sc.n), v);
      if constexpr (D == 3) {
        reinterpret_cast<float4 *>(s_v)[i] = make_float4(v[0], v[1], v[2], 0.0f);
      } else {
#pragma unroll
        for (int a = 0; a < D; ++a) s_v[a * LDS_NODES + i] = v[a];
      }
    }
    __syncthreads();
  }
  float ctl_val[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // CTL: new x and v of this lane
  bool ctl_have = false;
  auto body = [&]() {
  if (!ok) {
    float F[D * D];
    load_mat<D>(A.s.F, A.ld, p, F);
    // keep the output defined (the call reports the error)
    float z[D * D] = {};
    store_vec<D>(A.out.x, A.ld, p, xp);
    store_vec<D>(A.out.v, A.ld, p, z);
    store_mat<D>(A.out.C, A.ld, p, z);
    store_mat<D>(A.out.F, A.ld, p, F);
    if (eb) atomicOr(A.err, eb);
    return;
  }
  float w[D][3];
#pragma unroll
  for (int a = 0; a < D; ++a) bspline_w(f[a], w[a]);
  float vn[D] = {};
  float B[D * D] = {};  // sum_i N v_i (x_i - x_p)^T / dx
  const int lbase = box.lds ? box_index<D>(box, base) : 0;
  const int gbase = sc.g_off + node_index<D>(base, sc.n);
  if constexpr (D == 2) {
#pragma unroll
    for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
      for (int o1 = 0; o1 < 3; ++o1) {
        const float N = w[0][o0] * w[1][o1];
        const float d0 = (float)o0 - f[0], d1 = (float)o1 - f[1];
        float vi[2];
        if (box.lds) {
          const int li = lbase + o0 * box.e[1] + o1;
          vi[0] = s_v[li];
          vi[1] = s_v[LDS_NODES + li];
        } else {
          vel((int)(gbase - sc.g_off) + o0 * sc.n + o1, vi);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const float Nv = N * vi[a];
          vn[a] += Nv;
          B[a * 2 + 0] += Nv * d0;
          B[a * 2 + 1] += Nv * d1;
        }
      }
  } else {
    float Bm[3][3];
    if (box.lds) {  // (uniform over the workgroup)
      const float4 *s4 = reinterpret_cast<const float4 *>(s_v);
      g2p_sums3(w, f, [&](int o0, int o1, int o2, float *v) {
        const float4 n4 = s4[lbase + (o0 * box.e[1] + o1) * box.e[2] + o2];
        v[0] = n4.x;
        v[1] = n4.y;
        v[2] = n4.z;
      }, vn, Bm);
    } else {
      g2p_sums3(w, f, [&](int o0, int o1, int o2, float *v) {
        vel((int)(gbase - sc.g_off) + (o0 * sc.n + o1) * sc.n + o2, v);
      }, vn, Bm);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) B[a * 3 + b] = Bm[a][b];
  }
  // F is loaded after the stencil loop so it is not live across it
  float F[D * D];
  load_mat<D>(A.s.F, A.ld, p, F);
  // C' = (4/dx^2) sum N v_i (x_i - x_p)^T,  (x_i - x_p) = (o - f) dx
  const float cs = sc.Dinv * sc.dx;
  float Cn[D * D], Fn[D * D], xn[D];
#pragma unroll
  for (int k = 0; k < D * D; ++k) Cn[k] = cs * B[k];
  // F' = (I + dt C') F
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      float s = F[a * D + b];
#pragma unroll
      for (int g = 0; g < D; ++g) s += sc.dt * Cn[a * D + g] * F[g * D + b];
      Fn[a * D + b] = s;
    }
  // x' = x + dt v'
#pragma unroll
  for (int a = 0; a < D; ++a) xn[a] = xp[a] + sc.dt * vn[a];
  if (!(finite_all(xn, D) && finite_all(vn, D) && finite_all(Cn, D * D) &&
        finite_all(Fn, D * D)))
    eb |= EB_NONFINITE;
  store_vec<D>(A.out.x, A.ld, p, xn);
  store_vec<D>(A.out.v, A.ld, p, vn);
  store_mat<D>(A.out.C, A.ld, p, Cn);
  store_mat<D>(A.out.F, A.ld, p, Fn);
  if (eb) atomicOr(A.err, eb);
  if constexpr (CTL) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      ctl_val[a] = xn[a];
      ctl_val[D + a] = vn[a];
    }
    ctl_have = true;
  }
  };  // body
  if constexpr (!CTL) {
    if (active) body();
  } else {
    if (active) body();
    const int c = ctl_have ? A.ctl_comp[p] : -1;
    ctl_wave_add<D>(c, ctl_val, s_ctl[t >> 6]);
    __syncthreads();
    for (int i = t; i < A.ctl_nzs; i += CH)
      A.ctl_partial[(int64_t)i * A.ctl_rows + chunk] =
          (s_ctl[0][i] + s_ctl[1][i]) + (s_ctl[2][i] + s_ctl[3][i]);
  }
}

// ---------------------------------------------------------------------------
// reverse R1: adjoint of G2P, a particle -> grid scatter (supplement A-C)
// ---------------------------------------------------------------------------

template <int D>
__global__ __launch_bounds__(CH) void k_adj_scatter(AdjScatterArgs A) {
  __shared__ float s_grid[D * LDS_NODES];
  const Chunk ch = A.chunks[xcd_block_id()];
  const DevScene sc = A.scenes[ch.scene];
  const int t = threadIdx.x;
  const bool active = t < ch.count;
  const int p = ch.start + t;
  unsigned eb = 0;
  float xp[D], f[D];
  int base[D];
  bool ok = false;
  if (active) {
    load_vec<D>(A.s.x, A.ld, p, xp);
    ok = stencil_base<D>(xp, sc, base, f, eb);
  }
  const Box<D> box = chunk_box<D>(ok, base);
  float w[D][3], c0[D], Cdx[D][D];
  if (ok) {
    AdjScatterIn<D> in;
    adj_scatter_load<D>(A, p, in);
    adj_scatter_particle<D>(A, sc, in, f, w, c0, Cdx);
  }
  if (box.lds) {
    for (int i = t; i < D * LDS_NODES; i += CH) s_grid[i] = 0.0f;
    __syncthreads();
  }
  if (ok) {
    if (box.lds) {
      const int lbase = box_index<D>(box, base);
      scatter_stencil<D, false>(w, 0.0f, c0, Cdx,
                                [&](int o0, int o1, int o2, const float *val) {
        const int li = D == 2 ? lbase + o0 * box.e[1] + o1
                              : lbase + (o0 * box.e[1] + o1) * box.e[2] + o2;
#pragma unroll
        for (int c = 0; c < D; ++c) lds_add(&s_grid[c * LDS_NODES + li], val[c]);
      });
    } else {
      const int64_t gbase = sc.g_off + node_index<D>(base, sc.n);
      scatter_stencil<D, false>(w, 0.0f, c0, Cdx,
                                [&](int o0, int o1, int o2, const float *val) {
        add_global<D, 0>(nullptr, A.vbar, A.G,
                         stencil_gindex<D>(gbase, sc.n, o0, o1, o2), val);
      });
    }
  }
  if (box.lds) {
    __syncthreads();
    for (int i = t; i < box.vol; i += CH) {
      float v[D];
      bool nz = false;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        v[a] = s_grid[a * LDS_NODES + i];
        nz = nz || v[a] != 0.0f;
      }
      if (nz) {
        const int64_t gi = sc.g_off + box_node<D>(box, i, sc.n);
#pragma unroll
        for (int a = 0; a < D; ++a) gmem_add(&A.vbar[a * A.G + gi], v[a]);
      }
    }
  }
}

// Tile version of the adjoint scatter (binned particles); boxes carry d
// channels in slots 0..d-1 of the (d+1)-channel partial buffer.
template <int D, int B>
__global__ __launch_bounds__(256) void k_adj_scatter_tile(AdjScatterArgs A) {
  constexpr int S = TileBox<B>::S;
  constexpr int SV = D == 2 ? S * S : S * S * S;
  __shared__ float s_grid[D * SV];
  const int tile = blockIdx.x;
  const int cnt = A.tiles.cnt[tile];
  if (cnt == 0) return;
  const DevScene sc = A.scenes[A.tiles.scene[tile]];
  int org[D];
  tile_origin<D, B>(tile - sc.tile_off, sc.nt, org);
  const int t = threadIdx.x;
  for (int i = t; i < D * SV; i += 256) s_grid[i] = 0.0f;
  __syncthreads();
  unsigned eb = 0;
  const int start = A.tiles.start[tile];
  for (int j = t; j < cnt; j += 256) {
    const int p = start + j;
    float xp[D], f[D];
    int base[D];
    AdjScatterIn<D> in;
    load_vec<D>(A.s.x, A.ld, p, xp);
    adj_scatter_load<D>(A, p, in);
    if (!stencil_base<D>(xp, sc, base, f, eb)) continue;
    float w[D][3], c0[D], Cdx[D][D];
    adj_scatter_particle<D>(A, sc, in, f, w, c0, Cdx);
    int l[D];
    bool inbox = true;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      l[a] = base[a] - org[a];
      inbox = inbox && l[a] >= 0 && l[a] <= S - 3;
    }
    if (inbox) {
      const int lbase = D == 2 ? l[0] * S + l[1] : (l[0] * S + l[1]) * S + l[2];
      scatter_stencil<D, false>(w, 0.0f, c0, Cdx,
                                [&](int o0, int o1, int o2, const float *val) {
        const int li = D == 2 ? lbase + o0 * S + o1 : lbase + (o0 * S + o1) * S + o2;
#pragma unroll
        for (int c = 0; c < D; ++c) lds_add(&s_grid[c * SV + li], val[c]);
      });
    } else {
      const int64_t gbase = sc.g_off + node_index<D>(base, sc.n);
      scatter_stencil<D, false>(w, 0.0f, c0, Cdx,
                                [&](int o0, int o1, int o2, const float *val) {
        add_global<D, 0>(nullptr, A.vbar, A.G,
                         stencil_gindex<D>(gbase, sc.n, o0, o1, o2), val);
      });
    }
  }
  if (eb) atomicOr(A.err, eb);
  __syncthreads();
  float *dst = A.tiles.part + (int64_t)tile * (D + 1) * SV;
  for (int i = t; i < D * SV; i += 256)
    dst[i] = s_grid[(i / SV) * SV + box_node_at<D, B>(i % SV)];
}

// ---------------------------------------------------------------------------
// reverse R2: adjoint of the grid operations (supplement D-E)
// ---------------------------------------------------------------------------

template <int D>
__global__ __launch_bounds__(256) void k_adj_grid(AdjGridArgs A) {
  const GridBlock gb = A.blocks[xcd_block_id()];
  if ((int)threadIdx.x >= gb.count) return;
  const DevScene sc = A.scenes[gb.scene];
  const int li = gb.start + threadIdx.x;
  const int64_t gi = sc.g_off + li;
  const float m = A.gm[gi];
  const bool wall = is_wall<D>(li, sc.n, sc.wall);
  float vb[D], pb[D], v[D];
  bool nz = false;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    vb[a] = A.vbar[a * A.G + gi];
    nz = nz || vb[a] != 0.0f;
  }
  if (A.part) {
    const bool covered =
        add_tile_boxes_any<D, D>(A.B, sc, li, A.tile_cnt, A.part, D + 1, 0, vb);
    if (!covered && !nz && !(m > 0.0f)) return;  // untouched node (see k_grid)
  }
  float mb = 0.0f;
  if (m > 0.0f) {
    const float im = 1.0f / m;
    float vhat[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      vhat[a] = A.gp[a * A.G + gi] / m;  // before gravity (E)
      v[a] = vhat[a] + sc.dt * sc.g[a];
    }
    // wall nodes: v after the condition, dL/dv before it (sticky: 0; (L))
    if (wall) wall_bc_bwd<D>(sc, li, v, vb);
    float dot = 0.0f;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      pb[a] = vb[a] * im;                // (D)
      dot += vhat[a] * vb[a];
    }
    mb = -dot * im;                      // (E)
  } else {
#pragma unroll
    for (int a = 0; a < D; ++a) v[a] = pb[a] = 0.0f;
  }
#pragma unroll
  for (int a = 0; a < D; ++a) {
    A.pbar[a * A.G + gi] = pb[a];
    A.gv[a * A.G + gi] = v[a];
  }
  A.mbar[gi] = mb;
  if (nz) {
#pragma unroll
    for (int a = 0; a < D; ++a) A.vbar[a * A.G + gi] = 0.0f;
  }
}

// Adjoint grid operations over node tiles (see k_adj_grid and k_grid_nt).
template <int D>
__device__ __forceinline__ void adj_grid_nt_item(const AdjGridArgs &A, int ntg) {
  constexpr int B = D == 2 ? 8 : 4;
  constexpr int S = TileBox<B>::S, SV = D == 2 ? S * S : S * S * S;
  int li;
  int64_t gi;
  float vb[D];
  bool nz = false;
  float m;
  DevScene sc;
  bool from_cand = false;
  if constexpr (D == 3) {
    if (A.nt_cand) {
      // the box loads go out with the scene and flag loads (candidate table)
      from_cand = true;
      float val[8][3];
      const bool any = nt_cand_boxes<3>(A.nt_cand, A.part, ntg, val);
      const bool dirty = A.nt_dirty[ntg] != 0;
      if (!any && !dirty) return;
      sc = A.scenes[A.nt_scene[ntg]];
      if (!nt_node(sc, ntg, &li)) return;
      gi = sc.g_off + li;
#pragma unroll
      for (int a = 0; a < D; ++a) vb[a] = 0.0f;
      if (dirty) {
#pragma unroll
        for (int a = 0; a < D; ++a) {
          vb[a] = A.vbar[a * A.G + gi];
          nz = nz || vb[a] != 0.0f;
        }
      }
      m = A.gm[gi];
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int c = 0; c < D; ++c) vb[c] += val[k][c];
    }
  }
  if (!from_cand) {
    sc = A.scenes[A.nt_scene[ntg]];
    const NodeTile<D, B> nt = node_tile<D, B>(sc, ntg - sc.nt_off, A.tile_cnt);
    const bool dirty = A.nt_dirty[ntg] != 0;
    if ((!nt.any && !dirty) || !nt.valid) return;
    li = nt.li;
    gi = sc.g_off + li;
#pragma unroll
    for (int a = 0; a < D; ++a) vb[a] = 0.0f;
    if (dirty) {
#pragma unroll
      for (int a = 0; a < D; ++a) {
        vb[a] = A.vbar[a * A.G + gi];
        nz = nz || vb[a] != 0.0f;
      }
    }
    m = A.gm[gi];
    float val[NodeTile<D, B>::K][D];
#pragma unroll
    for (int k = 0; k < NodeTile<D, B>::K; ++k)
      if (nt.nz[k] && nt.cov[k]) {
        const float *bx = A.part + (int64_t)nt.tile[k] * (D + 1) * SV + box_pos<D, B>(nt.loc[k]);
#pragma unroll
        for (int c = 0; c < D; ++c) val[k][c] = bx[c * SV];
      }
#pragma unroll
    for (int k = 0; k < NodeTile<D, B>::K; ++k)
      if (nt.nz[k] && nt.cov[k]) {
#pragma unroll
        for (int c = 0; c < D; ++c) vb[c] += val[k][c];
      }
  }
  const bool wall = is_wall<D>(li, sc.n, sc.wall);
  float pb[D], v[D];
  float mb = 0.0f;
  if (m > 0.0f) {
    const float im = 1.0f / m;
    float vhat[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      vhat[a] = A.gp[a * A.G + gi] / m;  // before gravity (E)
      v[a] = vhat[a] + sc.dt * sc.g[a];
    }
    // wall nodes: v after the condition, dL/dv before it (sticky: 0; (L))
    if (wall) wall_bc_bwd<D>(sc, li, v, vb);
    float dot = 0.0f;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      pb[a] = vb[a] * im;                // (D)
      dot += vhat[a] * vb[a];
    }
    mb = -dot * im;                      // (E)
  } else {
#pragma unroll
    for (int a = 0; a < D; ++a) v[a] = pb[a] = 0.0f;
  }
#pragma unroll
  for (int a = 0; a < D; ++a) {
    A.pbar[a * A.G + gi] = pb[a];
    A.gv[a * A.G + gi] = v[a];
  }
  A.mbar[gi] = mb;
  if (nz) {
#pragma unroll
    for (int a = 0; a < D; ++a) A.vbar[a * A.G + gi] = 0.0f;
  }
}

template <int D, bool P>
__global__ __launch_bounds__(64) void k_adj_grid_nt(AdjGridArgs A) {
  for_items(A.n_nt, P, [&](int ntg) { adj_grid_nt_item<D>(A, ntg); });
}

// ---------------------------------------------------------------------------
// reverse R3: adjoint of P2G and of the particle update, a grid -> particle
// gather (supplement F-K)
// ---------------------------------------------------------------------------

// Node record of the adjoint gather: dL/dp (d), dL/dm, v (d), padded to 8
// floats, so a node is two 16-byte LDS reads (k_adj_gather keeps the two
// halves in separate arrays: a 16-byte node stride spreads the lanes of a
// wave over more LDS banks than a 32-byte one).
struct __align__(16) AdjNode {
  float4 a;  // pbar0, pbar1, pbar2 (or 0), mbar      (2D: pbar0, pbar1, 0, mbar)
  float4 b;  // v0, v1, v2 (or 0), unused
};

template <int D, typename Args>
__device__ __forceinline__ AdjNode adj_node_global(const Args &A, int64_t gi) {
  AdjNode r;
  r.a.x = A.pbar[gi];
  r.a.y = A.pbar[A.G + gi];
  r.a.z = D == 3 ? A.pbar[2 * A.G + gi] : 0.0f;
  r.a.w = A.mbar[gi];
  r.b.x = A.gv[gi];
  r.b.y = A.gv[A.G + gi];
  r.b.z = D == 3 ? A.gv[2 * A.G + gi] : 0.0f;
  r.b.w = 0.0f;
  return r;
}

// One particle's reverse of substep n once the scatter and grid reverses are
// done (supplement (F)-(K)).  In: the stencil fraction f of x^n, state n
// (v, C, F), the adjoint of state n+1 (gx1, gv1, gC1, gF1) and the
// particle's actuation; node(o0, o1, o2, nd) fetches the record (dL/dp_i,
// dL/dm_i, v_i) of stencil node base + o.  F^n and dL/dF^{n+1} are used
// again after the stencil loop; unpark(F, gF1) brings them back there (from
// LDS or a second read) so that they need not stay in registers across it.
// Out: xvc(ok, xb, vb, Cb) as soon as the x, v, C adjoints of state n are
// final, then fout(ok, Fb) with the F adjoint; sb_act += (K) for an actuated
// particle.  PM: pm_mass(ok, Nmb, Spb, Gb) and pm_stress(ok, Ptb, F, S,
// inner) hand over what the per-particle material gradients need.  MBS:
// the records carry m_p dL/dm_i (one scene-wide m_p, scaled once per staged
// node) in place of dL/dm_i.  ok is false (and eb set) when F^n is
// inverted; it is also returned.
template <int D, bool PM, bool MBS = false, typename Node, typename Unpark, typename XVC,
          typename FOut, typename PmMass, typename PmStress>
__device__ __forceinline__ bool adj_gather_particle(
    const DevScene &sc, const Mat &m, const float *f, const float *v, const float *C,
    const float *F0, const float *gx1, const float *gv1, const float *gC1,
    const float *gF10, float s_act, bool has_act, Node &&node, Unpark &&unpark,
    XVC &&xvc, FOut &&fout, PmMass &&pm_mass, PmStress &&pm_stress, unsigned &eb,
    float &sb_act) {
  // --- quantities live across the stencil loop ---------------------------
  float w[D][3], dw[D][3];
  // vt + (4/dx^2) Ct (x_i - x_p) = cV + CdxD o  (v-term and C-term of (J))
  float cV[D], CdxD[D][D];
  float cq[D], Gdx[D][D];  // m v + G (x_i - x_p) = cq + Gdx o
  bool ok;
  {
    Stress<D> S;
    ok = stress<D>(sc, m, F0, s_act, has_act, S, eb);
    float G[D * D];
    affine_G<D>(sc, m, S.Pt, F0, C, G);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      float s1 = gv1[a] + sc.dt * gx1[a];  // (A) vt
      float s2 = m.mp * v[a];
#pragma unroll
      for (int b = 0; b < D; ++b) {
        float ct = 0.0f;  // (B) Ct = gC1 + dt gF1 F^T
#pragma unroll
        for (int g = 0; g < D; ++g) ct += gF10[a * D + g] * F0[b * D + g];
        CdxD[a][b] = (gC1[a * D + b] + sc.dt * ct) * (sc.dx * sc.Dinv);
        Gdx[a][b] = G[a * D + b] * sc.dx;
        s1 -= CdxD[a][b] * f[b];
        s2 -= Gdx[a][b] * f[b];
      }
      cV[a] = s1;
      cq[a] = s2;
    }
  }
#pragma unroll
  for (int a = 0; a < D; ++a) {
    bspline_w(f[a], w[a]);
    bspline_dw(f[a], sc.inv_dx, dw[a]);
  }
  // Go = sum N p_i o^T (dL/dG = (Go - Spb f^T) dx after the loop);
  // Co = sum N v_i o^T gives C^{n+1} = (4/dx^2) dx (Co - Sv f^T), the G2P
  // of this substep, from the same node velocities
  float xb[D], Spb[D] = {}, Sv[D] = {}, Gb[D * D] = {}, Co[D * D] = {};
#pragma unroll
  for (int a = 0; a < D; ++a) xb[a] = gx1[a];  // (J) direct term dL/dx^{n+1}
  float Nmb = 0.0f;  // PM: sum N dL/dm_i
  auto add_node = [&](const AdjNode &nd, float N, const float *gN, const float *o) {
    const float pb[3] = {nd.a.x, nd.a.y, nd.a.z};
    const float vi[3] = {nd.b.x, nd.b.y, nd.b.z};
    float s_all = MBS ? nd.a.w : m.mp * nd.a.w;  // (J) m-term
    if constexpr (PM) Nmb += N * nd.a.w;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      float cv = cV[a], q = cq[a];
#pragma unroll
      for (int b = 0; b < D; ++b) {
        if (o[b] != 0.0f) {  // constant after unrolling; zero terms left out
          cv += CdxD[a][b] * o[b];
          q += Gdx[a][b] * o[b];
        }
      }
      // (J) v-term and C-term (N parts), p-term (N part)
      s_all += vi[a] * cv + pb[a] * q;
      const float Npb = N * pb[a], Nv = N * vi[a];
      Spb[a] += Npb;  // (F), and the delta part of the (J) p-term
      Sv[a] += Nv;    // delta part of the (J) C-term
#pragma unroll
      for (int b = 0; b < D; ++b) {
        if (o[b] != 0.0f) {
          Gb[a * D + b] += Npb * o[b];
          Co[a * D + b] += Nv * o[b];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < D; ++c) xb[c] += gN[c] * s_all;
  };
  if constexpr (D == 2) {
#pragma unroll
    for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
      for (int o1 = 0; o1 < 3; ++o1) {
        const float N = w[0][o0] * w[1][o1];
        const float gN[2] = {dw[0][o0] * w[1][o1], w[0][o0] * dw[1][o1]};
        const float o[2] = {(float)o0, (float)o1};
        AdjNode nd;
        node(o0, o1, 0, nd);
        add_node(nd, N, gN, o);
      }
  } else {
    // rows of the stencil are not unrolled: one row of node records in
    // flight instead of all 27 keeps the register count near the bound.
    // Within a row (o0, o1) only o2 varies, so the o0 and o1 columns of Go
    // and Co take the row's sums R = sum N p_i and Rv = sum N v_i once per
    // row, and Spb, Sv add the row sums.
#pragma unroll 1
    for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll 1
      for (int o1 = 0; o1 < 3; ++o1) {
        const float w01 = w[0][o0] * w[1][o1];
        const float d01 = dw[0][o0] * w[1][o1];
        const float w0d1 = w[0][o0] * dw[1][o1];
        const float fo0 = (float)o0, fo1 = (float)o1;
        float cv0[3], q0[3];  // cV + CdxD (o0, o1, 0), cq + Gdx (o0, o1, 0)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          cv0[a] = cV[a] + CdxD[a][0] * fo0 + CdxD[a][1] * fo1;
          q0[a] = cq[a] + Gdx[a][0] * fo0 + Gdx[a][1] * fo1;
        }
        float R[3] = {}, Rv[3] = {};
#pragma unroll
        for (int o2 = 0; o2 < 3; ++o2) {
          const float N = w01 * w[2][o2];
          const float gN[3] = {d01 * w[2][o2], w0d1 * w[2][o2], w01 * dw[2][o2]};
          AdjNode nd;
          node(o0, o1, o2, nd);
          const float pb[3] = {nd.a.x, nd.a.y, nd.a.z};
          const float vi[3] = {nd.b.x, nd.b.y, nd.b.z};
          float s_all = MBS ? nd.a.w : m.mp * nd.a.w;  // (J) m-term
          if constexpr (PM) Nmb += N * nd.a.w;
          const float No2 = N * (float)o2;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            // (J) v-term and C-term (N parts), p-term (N part)
            float cv = cv0[a], q = q0[a];
            if (o2 != 0) {
              cv += CdxD[a][2] * (float)o2;
              q += Gdx[a][2] * (float)o2;
            }
            s_all += vi[a] * cv + pb[a] * q;
            R[a] = fmaf(N, pb[a], R[a]);
            Rv[a] = fmaf(N, vi[a], Rv[a]);
            if (o2 != 0) {
              Gb[a * 3 + 2] = fmaf(No2, pb[a], Gb[a * 3 + 2]);
              Co[a * 3 + 2] = fmaf(No2, vi[a], Co[a * 3 + 2]);
            }
          }
#pragma unroll
          for (int c = 0; c < 3; ++c) xb[c] += gN[c] * s_all;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          Spb[a] += R[a];  // (F), and the delta part of the (J) p-term
          Sv[a] += Rv[a];  // delta part of the (J) C-term
          Gb[a * 3 + 0] += R[a] * fo0;
          Gb[a * 3 + 1] += R[a] * fo1;
          Co[a * 3 + 0] += Rv[a] * fo0;
          Co[a * 3 + 1] += Rv[a] * fo1;
        }
      }
  }
  // (J) delta parts: -sum N [ (4/dx^2) Ct^T v_i + G^T p_i ],
  // with Ct = Cdx / dx and G = Gdx / dx
#pragma unroll
  for (int c = 0; c < D; ++c) {
    float s = 0.0f;
#pragma unroll
    for (int a = 0; a < D; ++a) s += CdxD[a][c] * Sv[a] + Gdx[a][c] * Spb[a];
    xb[c] -= s * sc.inv_dx;
  }
  float C1[D * D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      Gb[a * D + b] -= Spb[a] * f[b];
      C1[a * D + b] = (sc.Dinv * sc.dx) * (Co[a * D + b] - Sv[a] * f[b]);
    }
  // --- after the loop: F^n and dL/dF^{n+1} back, the stress again ----------
  // (the compiler barrier keeps the pre-loop copies from staying live across
  // the stencil loop)
  asm volatile("" ::: "memory");
  float F[D * D], gF1[D * D];
  unpark(F, gF1);
  Stress<D> S;
  unsigned eb2 = 0;
  stress<D>(sc, m, F, s_act, has_act, S, eb2);
  float vb[D], Cb[D * D], Ptb[D * D], Fb[D * D];
#pragma unroll
  for (int a = 0; a < D; ++a) vb[a] = m.mp * Spb[a];  // (F)
#pragma unroll
  for (int k = 0; k < D * D; ++k) {
    Gb[k] *= sc.dx;        // dL/dG = sum N p_i (x_i - x_p)^T
    Cb[k] = m.mp * Gb[k];  // (I)
  }
  if constexpr (PM) pm_mass(ok, Nmb, Spb, Gb);
  if (!(finite_all(xb, D) && finite_all(vb, D) && finite_all(Cb, D * D)))
    eb |= EB_NONFINITE;
  // x, v and C adjoints are final
  xvc(ok, xb, vb, Cb);
  // (G) dL/dP_t = kG dL/dG F
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      float s = 0.0f;
#pragma unroll
      for (int g = 0; g < D; ++g) s += Gb[a * D + g] * F[g * D + b];
      Ptb[a * D + b] = sc.kG * s;
    }
  // (H) update term (I + dt C^{n+1})^T dL/dF^{n+1}
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      float s = gF1[a * D + b];
#pragma unroll
      for (int g = 0; g < D; ++g) s += sc.dt * C1[g * D + a] * gF1[g * D + b];
      Fb[a * D + b] = s;
    }
  // (H) G-term kG dL/dG^T P_t and actuation term dL/dP_t sigma^T
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      float s = 0.0f;
#pragma unroll
      for (int g = 0; g < D; ++g) s += Gb[g * D + a] * S.Pt[g * D + b];
      Fb[a * D + b] += sc.kG * s + Ptb[a * D + b] * S.sigma[b];
    }
  // (H) elastic term: mu Ptb + (mu - la lnJ) F^-T Ptb^T F^-T
  //                  + la <Ptb, F^-T> F^-T
  float inner = 0.0f, T1[D * D];
#pragma unroll
  for (int k = 0; k < D * D; ++k) inner += Ptb[k] * S.FiT[k];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      float s = 0.0f;  // (F^-T Ptb^T)_ab
#pragma unroll
      for (int g = 0; g < D; ++g) s += S.FiT[a * D + g] * Ptb[b * D + g];
      T1[a * D + b] = s;
    }
  const float cmu = m.mu - m.la * S.lnJ;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      float s = 0.0f;
#pragma unroll
      for (int g = 0; g < D; ++g) s += T1[a * D + g] * S.FiT[g * D + b];
      Fb[a * D + b] += m.mu * Ptb[a * D + b] + cmu * s + m.la * inner * S.FiT[a * D + b];
    }
  if constexpr (PM) pm_stress(ok, Ptb, F, S, inner);
  // (K) dL/dsigma_aa = (F^T dL/dP_t)_aa;  s-bar = sum_a axis_a sigma-bar_aa
  if (has_act) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      float s = 0.0f;
#pragma unroll
      for (int g = 0; g < D; ++g) s += F[g * D + a] * Ptb[g * D + a];
      sb_act += sc.axis[a] * s;
    }
  }
  if (!finite_all(Fb, D * D)) eb |= EB_NONFINITE;
  fout(ok, Fb);
  return ok;
}

// Launched for three waves per SIMD (at most 168 VGPRs): with F and dL/dF
// parked in LDS across the stencil loop the 3D kernel fits without spills.
// PM: the context has per-particle materials (mu, la, m_p per particle);
// their gradients dL/dmu_p, dL/dla_p, dL/dm_p are added to A.gmat.
template <int D, bool PM>
__global__ __launch_bounds__(CH, 3) void k_adj_gather(AdjGatherArgs A) {
  __shared__ float4 s_na[LDS_NODES], s_nb[LDS_NODES];  // AdjNode halves a, b
  __shared__ double s_act[LDS_ACT];
  // F^n and dL/dF^{n+1} of each thread, kept for the post-loop algebra
  __shared__ float s_keep[D == 3 ? 2 * D * D * CH : 1];
  const Chunk ch = A.chunks[xcd_block_id()];
  const DevScene sc = A.scenes[ch.scene];
  const int t = threadIdx.x;
  const bool active = t < ch.count;
  const int p = ch.start + t;
  if (A.n >= sc.t_end) {
    // past the scene's horizon the substep is the identity: the adjoint is
    // carried over and adds nothing to dL/ds or the material gradients
    if (active) {
      float a[D * D];
      load_vec<D>(A.g1.x, A.ld, p, a);
      store_vec<D>(A.g0.x, A.ld, p, a);
      load_vec<D>(A.g1.v, A.ld, p, a);
      store_vec<D>(A.g0.v, A.ld, p, a);
      load_mat<D>(A.g1.C, A.ld, p, a);
      store_mat<D>(A.g0.C, A.ld, p, a);
      load_mat<D>(A.g1.F, A.ld, p, a);
      store_mat<D>(A.g0.F, A.ld, p, a);
      if (A.sb_part) A.sb_part[p] = 0.0f;
    }
    return;
  }
  unsigned eb = 0;
  float xp[D], f[D];
  int base[D];
  bool ok = false;
  // the particle's streams are requested before the node staging and its
  // barriers, so their latency overlaps the staging
  float v[D], C[D * D], F[D * D], gx1[D], gv1[D], gC1[D * D], gF1[D * D];
  int j_act = -1;
  if (active) {
    load_vec<D>(A.s.x, A.ld, p, xp);
    load_vec<D>(A.s.v, A.ld, p, v);
    load_mat<D>(A.s.C, A.ld, p, C);
    load_mat<D>(A.s.F, A.ld, p, F);
    load_vec<D>(A.g1.x, A.ld, p, gx1);
    load_vec<D>(A.g1.v, A.ld, p, gv1);
    load_mat<D>(A.g1.C, A.ld, p, gC1);
    load_mat<D>(A.g1.F, A.ld, p, gF1);
    j_act = A.act_id[p];
    ok = stencil_base<D>(xp, sc, base, f, eb);
  }
  Mat m = scene_mat(sc);
  if (PM && active) m = particle_mat(A.mat, A.ld, sc, p);
  const Box<D> box = chunk_box<D>(ok, base);
  const bool act_lds = sc.n_act <= LDS_ACT && A.gact != nullptr;
  if (act_lds)
    for (int i = t; i < sc.n_act; i += CH) s_act[i] = 0.0;
  if (box.lds) {
    for (int i = t; i < box.vol; i += CH) {
      AdjNode r = adj_node_global<D>(A, sc.g_off + box_node<D>(box, i, sc.n));
      if constexpr (!PM) r.a.w *= sc.mp;  // m_p dL/dm_i, the (J) m-term's factor
      s_na[i] = r.a;
      s_nb[i] = r.b;
    }
  }
  __syncthreads();

  float sb_act = 0.0f;
  if (!ok) j_act = -1;
  if (ok) {
    const float s_act = j_act >= 0 ? A.act[sc.act_off + j_act] : 0.0f;
    if constexpr (D == 3) {
#pragma unroll
      for (int q = 0; q < D * D; ++q) {
        s_keep[q * CH + t] = F[q];
        s_keep[(D * D + q) * CH + t] = gF1[q];
      }
    }
    const int lbase = box.lds ? box_index<D>(box, base) : 0;
    const int64_t gbase = sc.g_off + node_index<D>(base, sc.n);
    ok = adj_gather_particle<D, PM, !PM>(
        sc, m, f, v, C, F, gx1, gv1, gC1, gF1, s_act, j_act >= 0,
        [&](int o0, int o1, int o2, AdjNode &nd) {
          if (box.lds) {
            const int li = D == 2 ? lbase + o0 * box.e[1] + o1
                                  : lbase + (o0 * box.e[1] + o1) * box.e[2] + o2;
            nd.a = s_na[li];
            nd.b = s_nb[li];
          } else {
            nd = adj_node_global<D>(A, D == 2 ? gbase + o0 * sc.n + o1
                                              : gbase + ((int64_t)o0 * sc.n + o1) * sc.n + o2);
            if constexpr (!PM) nd.a.w *= sc.mp;
          }
        },
        [&](float *Fr, float *gFr) {
          if constexpr (D == 3) {
#pragma unroll
            for (int q = 0; q < D * D; ++q) {
              Fr[q] = s_keep[q * CH + t];
              gFr[q] = s_keep[(D * D + q) * CH + t];
            }
          } else {
            load_mat<D>(A.s.F, A.ld, p, Fr);
            load_mat<D>(A.g1.F, A.ld, p, gFr);
          }
        },
        [&](bool okp, const float *xb, const float *vb, const float *Cb) {
          if (okp) {
            store_vec<D>(A.g0.x, A.ld, p, xb);
            store_vec<D>(A.g0.v, A.ld, p, vb);
            store_mat<D>(A.g0.C, A.ld, p, Cb);
          }
        },
        [&](bool okp, const float *Fb) {
          if (okp) store_mat<D>(A.g0.F, A.ld, p, Fb);
        },
        [&](bool okp, float Nmb, const float *Spb, const float *Gb) {
          // dL/dm_p = sum N [dL/dm_i + dL/dp_i . (v_p + C_p (x_i - x_p))]
          if (A.gmat && okp) {
            float vv[D], CC[D * D];
            load_vec<D>(A.s.v, A.ld, p, vv);
            load_mat<D>(A.s.C, A.ld, p, CC);
            float mbp = Nmb;
#pragma unroll
            for (int a = 0; a < D; ++a) mbp += vv[a] * Spb[a];
#pragma unroll
            for (int k = 0; k < D * D; ++k) mbp += CC[k] * Gb[k];
            A.gmat[2 * (int64_t)A.ld + p] += mbp;
          }
        },
        [&](bool okp, const float *Ptb, const float *Fr, const Stress<D> &S, float inner) {
          // dL/dmu_p = <dL/dP, F - F^-T>, dL/dla_p = ln J <dL/dP, F^-T>
          if (A.gmat && okp) {
            float mub = 0.0f;
#pragma unroll
            for (int k = 0; k < D * D; ++k) mub += Ptb[k] * (Fr[k] - S.FiT[k]);
            A.gmat[p] += mub;
            A.gmat[(int64_t)A.ld + p] += S.lnJ * inner;
          }
        },
        eb, sb_act);
  }
  if (active && !ok) {
    float z[D * D] = {};
    store_vec<D>(A.g0.x, A.ld, p, z);
    store_vec<D>(A.g0.v, A.ld, p, z);
    store_mat<D>(A.g0.C, A.ld, p, z);
    store_mat<D>(A.g0.F, A.ld, p, z);
  }
  if (eb) atomicOr(A.err, eb);
  if (A.sb_part && active) A.sb_part[p] = ok && j_act >= 0 ? sb_act : 0.0f;
  if (A.gact != nullptr) {
    if (act_lds) {
      if (ok && j_act >= 0)
        __hip_atomic_fetch_add(&s_act[j_act], (double)sb_act, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
      __syncthreads();
      for (int i = t; i < sc.n_act; i += CH)
        if (s_act[i] != 0.0) unsafeAtomicAdd(&A.gact[sc.act_off + i], s_act[i]);
    } else if (ok && j_act >= 0) {
      unsafeAtomicAdd(&A.gact[sc.act_off + j_act], (double)sb_act);
    }
  }
}

// The reverse of substep n's G2P/P2G gather fused with the adjoint scatter
// of substep n-1, in one pass over a tile (3D): the tile's box of the
// adjoint grid of substep n is staged in LDS, each thread runs the gather
// (supplement (F)-(K)) for its particles and writes the adjoint of state n,
// and hands that adjoint from registers to the scatter's record step of
// substep n-1 ((A)-(C) with x^{n-1}, F^{n-1}), so the adjoint of state n is
// not read back from HBM.  Particles whose stencil left the box read the
// adjoint grid from HBM (gather) or add to it with global atomics (scatter).
// F^n and dL/dF^{n+1} are read a second time after the stencil loop
// (cached), which keeps the kernel within three workgroups per CU.
template <int D, bool DET>
__global__ __launch_bounds__(256, 2) void k_adj_gather_scatter(AdjFusedArgs A) {
  static_assert(D == 3, "the fused reverse pass is built for 3D tiles");
  using SC = SortedCell<D>;
  constexpr int S = SC::S, SV = SC::SV, BC = SC::BC, B = SC::B;
  __shared__ SortedCellSmem<D, D, 2, false, false, DET> sm;
  __shared__ AdjNode s_n[SV];
  __shared__ double s_act[LDS_ACT];
  const int tile = A.tiles.list ? A.tiles.list[blockIdx.x] : blockIdx.x;
  if (A.tiles.cnt[tile] == 0) return;
  const DevScene sc = A.scenes[A.tiles.scene[tile]];
  const int t = threadIdx.x;
  int org[D];
  tile_origin<D, B>(tile - sc.tile_off, sc.nt, org);
  for (int i = t; i < SV; i += 256) {
    const int g[3] = {org[0] + i / (S * S), org[1] + (i / S) % S, org[2] + i % S};
    const bool in = g[0] >= 0 && g[0] < sc.n && g[1] >= 0 && g[1] < sc.n &&
                    g[2] >= 0 && g[2] < sc.n;
    AdjNode nd{};
    if (in) nd = adj_node_global<D>(A, sc.g_off + ((int64_t)g[0] * sc.n + g[1]) * sc.n + g[2]);
    s_n[i] = nd;
  }
  const bool act_lds = sc.n_act <= LDS_ACT && A.gact != nullptr;
  if (act_lds)
    for (int i = t; i < sc.n_act; i += 256) s_act[i] = 0.0;
  // (the scatter synchronises before its record step reads s_n and s_act)
  const Mat m = scene_mat(sc);
  auto part = [&](int p, int *base, float *f, float (&w)[D][3], float *c0,
                  float (&Cdx)[D][D], unsigned &eb) {
    // --- reverse of substep n: gather ------------------------------------
    float xn[D], fn[D], v[D], C[D * D], F[D * D], gx1[D], gv1[D], gC1[D * D], gF1[D * D];
    int bn[D];
    load_vec<D>(A.s.x, A.ld, p, xn);
    load_vec<D>(A.s.v, A.ld, p, v);
    load_mat<D>(A.s.C, A.ld, p, C);
    load_mat<D>(A.s.F, A.ld, p, F);
    load_vec<D>(A.g1.x, A.ld, p, gx1);
    load_vec<D>(A.g1.v, A.ld, p, gv1);
    load_mat<D>(A.g1.C, A.ld, p, gC1);
    load_mat<D>(A.g1.F, A.ld, p, gF1);
    const int j_act = A.act_id[p];
    bool ok = stencil_base<D>(xn, sc, bn, fn, eb);
    float vt[D], Cb[D * D], Fb[D * D];
    float sb_act = 0.0f;
    if (A.n >= sc.t_end) {
      // past the scene's horizon substep n is the identity: the adjoint of
      // state n+1 is carried over
      store_vec<D>(A.g0.x, A.ld, p, gx1);
      store_vec<D>(A.g0.v, A.ld, p, gv1);
      store_mat<D>(A.g0.C, A.ld, p, gC1);
      store_mat<D>(A.g0.F, A.ld, p, gF1);
#pragma unroll
      for (int a = 0; a < D; ++a) vt[a] = gv1[a] + sc.dt * gx1[a];
#pragma unroll
      for (int k = 0; k < D * D; ++k) {
        Cb[k] = gC1[k];
        Fb[k] = gF1[k];
      }
      if (A.sb_part) A.sb_part[p] = 0.0f;
      ok = true;
    } else if (ok) {
      int lb[D];
      bool inb = true;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        lb[a] = bn[a] - org[a];
        inb = inb && lb[a] >= 0 && lb[a] < BC;
      }
      const int lbase = (lb[0] * S + lb[1]) * S + lb[2];
      const int64_t gbase = sc.g_off + node_index<D>(bn, sc.n);
      const float s_n_act = j_act >= 0 ? A.act[sc.act_off + j_act] : 0.0f;
      ok = adj_gather_particle<D, false>(
          sc, m, fn, v, C, F, gx1, gv1, gC1, gF1, s_n_act, j_act >= 0,
          [&](int o0, int o1, int o2, AdjNode &nd) {
            nd = inb ? s_n[lbase + (o0 * S + o1) * S + o2]
                     : adj_node_global<D>(A, gbase + ((int64_t)o0 * sc.n + o1) * sc.n + o2);
          },
          [&](float *Fr, float *gFr) {
            load_mat<D>(A.s.F, A.ld, p, Fr);
            load_mat<D>(A.g1.F, A.ld, p, gFr);
          },
          [&](bool okp, const float *xb, const float *vb, const float *Cbar) {
            if (okp) {
              store_vec<D>(A.g0.x, A.ld, p, xb);
              store_vec<D>(A.g0.v, A.ld, p, vb);
              store_mat<D>(A.g0.C, A.ld, p, Cbar);
            }
            // (A) of substep n-1: dL/dv^n total = carried + dt dL/dx^n
#pragma unroll
            for (int a = 0; a < D; ++a) vt[a] = vb[a] + sc.dt * xb[a];
#pragma unroll
            for (int k = 0; k < D * D; ++k) Cb[k] = Cbar[k];
          },
          [&](bool okp, const float *Fbar) {
            if (okp) store_mat<D>(A.g0.F, A.ld, p, Fbar);
#pragma unroll
            for (int k = 0; k < D * D; ++k) Fb[k] = Fbar[k];
          },
          [](bool, float, const float *, const float *) {},
          [](bool, const float *, const float *, const Stress<D> &, float) {}, eb,
          sb_act);
      if (ok && j_act >= 0 && A.gact != nullptr) {
        if (act_lds)
          __hip_atomic_fetch_add(&s_act[j_act], (double)sb_act, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
        else
          unsafeAtomicAdd(&A.gact[sc.act_off + j_act], (double)sb_act);
      }
    }
    if (A.sb_part && A.n < sc.t_end) A.sb_part[p] = ok && j_act >= 0 ? sb_act : 0.0f;
    if (!ok) {
      float z[D * D] = {};
      store_vec<D>(A.g0.x, A.ld, p, z);
      store_vec<D>(A.g0.v, A.ld, p, z);
      store_mat<D>(A.g0.C, A.ld, p, z);
      store_mat<D>(A.g0.F, A.ld, p, z);
      return false;  // a zero adjoint adds nothing to substep n-1
    }
    // --- adjoint scatter of substep n-1 -----------------------------------
    if (A.n - 1 >= sc.t_end) return false;  // the identity past the horizon
    float xp[D], Fp[D * D];
    load_vec<D>(A.sp.x, A.ld, p, xp);
    if (!stencil_base<D>(xp, sc, base, f, eb)) return false;
    load_mat<D>(A.sp.F, A.ld, p, Fp);
    // (B): dL/dC^n total = carried + dt dL/dF^n F^{n-1 T}
    const float cs = sc.Dinv * sc.dx;
#pragma unroll
    for (int a = 0; a < D; ++a) bspline_w(f[a], w[a]);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      // (C): vt + (4/dx^2) Ct (x_i - x_p), x_i - x_p = (o - f) dx
      float s0 = vt[a];
#pragma unroll
      for (int b = 0; b < D; ++b) {
        float ct = 0.0f;
#pragma unroll
        for (int g = 0; g < D; ++g) ct += Fb[a * D + g] * Fp[b * D + g];
        Cdx[a][b] = cs * (Cb[a * D + b] + sc.dt * ct);
        s0 -= Cdx[a][b] * f[b];
      }
      c0[a] = s0;
    }
    return true;
  };
  // the scatter's cells come from x^{n-1} alone, before the gathers
  auto cell = [&](int p, int *base, unsigned &eb) {
    float xp[D], f[D];
    load_vec<D>(A.sp.x, A.ld, p, xp);
    return stencil_base<D>(xp, sc, base, f, eb);
  };
  sorted_cell_scatter<D, D, false, 2, false>(A, tile, sm, nullptr, A.vbar, part, cell);
  if (act_lds) {
    __syncthreads();
    for (int i = t; i < sc.n_act; i += 256)
      if (s_act[i] != 0.0) unsafeAtomicAdd(&A.gact[sc.act_off + i], s_act[i]);
  }
}

// ---------------------------------------------------------------------------
// binning (once per rollout): tile, rank within the cell, cell
// ---------------------------------------------------------------------------

template <int D>
__device__ __forceinline__ int ipow(int b) {
  return D == 2 ? b * b : b * b * b;
}

template <int D>
__global__ __launch_bounds__(256) void k_sort_count(SortArgs A) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= A.N) return;
  const DevScene sc = A.scenes[A.pscene[p]];
  float xp[D], f[D];
  int base[D];
  unsigned eb = 0;
  load_vec<D>(A.x, A.ld, p, xp);
  if (!stencil_base<D>(xp, sc, base, f, eb)) {
    atomicOr(A.err, eb);
    A.ptile[p] = -1;
    return;
  }
  const int TB = A.tile;
  const int nt = (sc.n - 2 + TB - 1) / TB;  // tiles per axis
  int tl = 0, cl = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    tl = tl * nt + base[a] / TB;
    cl = cl * TB + base[a] % TB;
  }
  const int tile = sc.tile_off + tl;
  const int rank = atomicAdd(&A.cell_cnt[(int64_t)tile * ipow<D>(TB) + cl], 1);
  // per-tile counts: the lanes of a wave mostly share a tile (particles in
  // tile order), so one atomic per distinct tile of the wave
  unsigned long long pending = __ballot(1);
  while (pending) {
    const int lead = __ffsll((long long)pending) - 1;
    const int lt = __shfl(tile, lead, 64);
    const unsigned long long same = __ballot(tile == lt) & pending;
    if ((int)(threadIdx.x & 63) == lead) atomicAdd(&A.tile_cnt[lt], __popcll(same));
    pending &= ~same;
  }
  A.ptile[p] = tile;
  A.pcell[p] = cl;
  A.prank[p] = rank;
}

// Position of a particle in tile order: all rank-0 particles of the tile (by
// cell), then all rank-1 particles, ...  Consecutive lanes hold distinct cells.
template <int D>
__global__ __launch_bounds__(256) void k_sort_place(SortArgs A,
                                                    const int *tile_start,
                                                    int *perm) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= A.N) return;
  const int tile = A.ptile[p];
  if (tile < 0) return;
  const int c = A.pcell[p], r = A.prank[p];
  const int cpt = ipow<D>(A.tile);
  const int *cnt = A.cell_cnt + (int64_t)tile * cpt;
  int pos = tile_start[tile];
  for (int k = 0; k < cpt; ++k) {
    const int nk = cnt[k];
    pos += min(nk, r) + ((k < c && nk > r) ? 1 : 0);
  }
  perm[pos] = p;
}

__global__ __launch_bounds__(256) void k_chunk_count(const int *tile_cnt,
                                                     int n, int *nch) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) nch[i] = (tile_cnt[i] + CH - 1) / CH;
}

__global__ __launch_bounds__(256) void k_nonempty_flag(const int *tile_cnt,
                                                       int n, int *flag) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) flag[i] = tile_cnt[i] > 0 ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_compact(const int *flag, const int *pos,
                                                 int n, int *list) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n && flag[i]) list[pos[i]] = i;
}

__global__ __launch_bounds__(256) void k_build_chunks(
    const int *tile_cnt, const int *tile_start, const int *chunk_start,
    const int *tile_scene, int n, Chunk *chunks) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int cnt = tile_cnt[i];
  const int c0 = chunk_start[i];
  for (int k = 0; k * CH < cnt; ++k) {
    Chunk c;
    c.scene = tile_scene[i];
    c.start = tile_start[i] + k * CH;
    c.count = min(CH, cnt - k * CH);
    c.pad = 0;
    chunks[c0 + k] = c;
  }
}

// Exclusive scan with one 1024-thread workgroup; out has n+1 entries.
__global__ __launch_bounds__(1024) void k_scan_i32(const int *in, int *out,
                                                   int n) {
  __shared__ int s[1024];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < n; base += 1024) {
    const int i = base + threadIdx.x;
    const int v = i < n ? in[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int add = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < n) out[i] = carry + s[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = carry;
}

__global__ __launch_bounds__(256) void k_permute_rows(const float *in,
                                                      float *out,
                                                      const int *perm, int N,
                                                      int ld, int ncomp,
                                                      int scatter) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const int q = perm[i];
  if ((unsigned)q >= (unsigned)N) return;  // never follow an invalid index
  for (int c = 0; c < ncomp; ++c) {
    if (scatter)
      out[(int64_t)c * ld + q] = in[(int64_t)c * ld + i];
    else
      out[(int64_t)c * ld + i] = in[(int64_t)c * ld + q];
  }
}

__global__ __launch_bounds__(256) void k_permute_i32(const int *in, int *out,
                                                     const int *perm, int N) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const int q = perm[i];
  out[i] = (unsigned)q < (unsigned)N ? in[q] : -1;  // never follow an invalid index
}

// ---------------------------------------------------------------------------
// fills, actuation-gradient store, sinusoid actuation bank
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t k = i; k < n; k += stride) p[k] = T(0);
}

// ---------------------------------------------------------------------------
// closed-loop controller a = tanh(W z + b) (section IV, Control)
// ---------------------------------------------------------------------------

constexpr int CTL_WG = 1024;      // workgroups of the controller kernels at most

// Sums of x and v over each component, one row of partial sums per
// workgroup (grid-stride over the particles).  Per wave, the lanes of one
// component at a time are reduced with a reduce-scatter butterfly (the 2d
// values padded to 8: 10 cross-lane steps instead of 6 per value), lane
// group v ending with the total of value v, which it adds to the wave's LDS
// row (entry 2 d c + a: x_a of component c, 2 d c + d + a: v_a).  Rows are
// stored entry-major so the reduction reads them contiguously.
template <int D>
__global__ __launch_bounds__(256) void k_ctl_partial(CtlArgs A, int n_rows) {
  __shared__ float s_w[4][CTL_MAX_NZS];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int nzs = 2 * D * A.n_comp;
  for (int i = lane; i < CTL_MAX_NZS; i += 64) s_w[wave][i] = 0.0f;
  for (int p0 = blockIdx.x * 256; p0 < A.N; p0 += n_rows * 256) {
    const int p = p0 + t;
    const bool in = p < A.N;
    // loads independent of the component id: one memory round trip
    const int c = in ? A.comp[p] : -1;
    float val[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) {
      val[a] = in ? A.x[a * A.ld + p] : 0.0f;
      val[D + a] = in ? A.v[a * A.ld + p] : 0.0f;
    }
    ctl_wave_add<D>(c, val, s_w[wave]);
  }
  __syncthreads();
  for (int i = t; i < nzs; i += 256)
    A.partial[(int64_t)i * n_rows + blockIdx.x] =
        (s_w[0][i] + s_w[1][i]) + (s_w[2][i] + s_w[3][i]);
}

// One workgroup per entry: the sum over the partial rows (FP64).  The last
// workgroup to finish forms z = [target, component means] and evaluates
// a = tanh(W z + b) (one wave per row).
__global__ __launch_bounds__(256) void k_ctl_reduce(CtlArgs A, int n_rows) {
  __shared__ double s_red[256];
  __shared__ bool s_last;
  __shared__ double s_z[CTL_MAX_NZS + 3];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, d = A.dim;
  const int nzs = 2 * d * A.n_comp;
  const int i = blockIdx.x;
  double acc = 0.0;
  for (int w = t; w < n_rows; w += 256) acc += (double)A.partial[(int64_t)i * n_rows + w];
  s_red[t] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) s_red[t] += s_red[t + s];
    __syncthreads();
  }
  if (t == 0) {
    A.sums[i] = s_red[0];
    __threadfence();
    s_last = atomicAdd(A.done, 1u) == (unsigned)(nzs - 1);
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  for (int k = t; k < A.nz; k += 256) {
    double zk;
    if (k < d) {
      zk = A.target[k];
    } else {
      const int c = (k - d) / (2 * d);
      zk = ((volatile double *)A.sums)[k - d] * (double)A.inv_cnt[c];
    }
    s_z[k] = zk;
    A.z[k] = (float)zk;
  }
  __syncthreads();
  // W z + b: one wave per row, lanes over z (nz <= 99 < 128)
  for (int j = wave; j < A.n_act; j += 4) {
    float x = 0.0f;
    if (lane < A.nz) x = A.W[j * A.nz + lane] * (float)s_z[lane];
    if (lane + 64 < A.nz) x += A.W[j * A.nz + lane + 64] * (float)s_z[lane + 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) A.act[j] = tanhf(A.b[j] + x);
  }
  if (t == 0) *A.done = 0u;  // for the next substep (stream-ordered)
}

// Reverse of the controller at one substep.  Every workgroup forms
// g = dL/ds (1 - a^2) and the state part of W^T g divided by each
// component's particle count, then adds it to the x and v adjoints of the
// component's particles (grid-stride); workgroup 0 also accumulates
// dL/dW += g z^T and dL/db += g.
__global__ __launch_bounds__(256) void k_ctl_adjoint(CtlAdjArgs A, int n_wg) {
  __shared__ double s_g[64];
  __shared__ float s_zs[CTL_MAX_NZS];
  const int t = threadIdx.x, d = A.dim, nzs = 2 * d * A.n_comp;
  for (int j = t; j < A.n_act; j += 256) {
    const double a = A.act[j];
    const double g = A.sbar[j] * (1.0 - a * a);
    s_g[j] = g;
    if (blockIdx.x == 0) A.gb[j] += g;
  }
  __syncthreads();
  if (blockIdx.x == 0)
    for (int e = t; e < A.n_act * A.nz; e += 256) {
      const int j = e / A.nz, k = e % A.nz;
      A.gW[e] += s_g[j] * (double)A.z[k];
    }
  for (int k = t; k < nzs; k += 256) {
    double s = 0.0;
#pragma unroll 8
    for (int j = 0; j < A.n_act; ++j) s += (double)A.W[j * A.nz + d + k] * s_g[j];
    s_zs[k] = (float)(s * (double)A.inv_cnt[k / (2 * d)]);
  }
  __syncthreads();
  for (int p = blockIdx.x * 256 + t; p < A.N; p += n_wg * 256) {
    const int c = A.comp[p];
    if (c < 0) continue;
    for (int a = 0; a < d; ++a) {
      A.gx[a * A.ld + p] += s_zs[2 * d * c + a];
      A.gv[a * A.ld + p] += s_zs[2 * d * c + d + a];
    }
  }
}

__global__ __launch_bounds__(256) void k_gact_store(const double *src,
                                                    float *dst, int64_t n,
                                                    int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float v = (float)src[i];
  dst[i] = accumulate ? dst[i] + v : v;
}

__global__ __launch_bounds__(256) void k_act_bank_fwd(int T, int n_act,
                                                      int n_freq, float dt,
                                                      const float *freq,
                                                      const float *amp,
                                                      const float *phase,
                                                      float *act) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= T * n_act) return;
  const int n = i / n_act, j = i % n_act;
  const double t = (double)n * (double)dt;
  double s = 0.0;
  for (int k = 0; k < n_freq; ++k)
    s += (double)amp[j * n_freq + k] *
         sin(2.0 * M_PI * (double)freq[k] * t + (double)phase[j * n_freq + k]);
  act[i] = (float)s;
}

// One workgroup per (j, k): reduce over the T steps.
__global__ __launch_bounds__(256) void k_act_bank_bwd(
    int T, int n_act, int n_freq, float dt, const float *freq,
    const float *amp, const float *phase, const float *g_act, float *g_amp,
    float *g_phase) {
  __shared__ double s_a[256], s_p[256];
  const int jk = blockIdx.x;
  const int j = jk / n_freq, k = jk % n_freq;
  double ga = 0.0, gp = 0.0;
  for (int n = threadIdx.x; n < T; n += 256) {
    const double th = 2.0 * M_PI * (double)freq[k] * ((double)n * (double)dt) +
                      (double)phase[jk];
    const double g = (double)g_act[(int64_t)n * n_act + j];
    ga += g * sin(th);
    gp += g * (double)amp[jk] * cos(th);
  }
  s_a[threadIdx.x] = ga;
  s_p[threadIdx.x] = gp;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s_a[threadIdx.x] += s_a[threadIdx.x + off];
      s_p[threadIdx.x] += s_p[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    g_amp[jk] = (float)s_a[0];
    g_phase[jk] = (float)s_p[0];
  }
}

inline int hip_rc(hipError_t e) { return e == hipSuccess ? 0 : -6; }

inline int blocks_for(int64_t n, int per = 256) {
  return (int)((n + per - 1) / per);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

#define MPM_LAUNCH(kernel, grid, block, st, ...)                       \
  do {                                                                 \
    if ((grid) > 0) {                                                  \
      hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, st,       \
                         __VA_ARGS__);                                 \
      return hip_rc(hipGetLastError());                                \
    }                                                                  \
    return 0;                                                          \
  } while (0)

int launch_p2g(int dim, const P2GArgs &a, hipStream_t st) {
  if (dim == 2) MPM_LAUNCH(k_p2g<2>, a.n_chunks, CH, st, a);
  MPM_LAUNCH(k_p2g<3>, a.n_chunks, CH, st, a);
}

bool tile_supported(int dim, int B) {
  return dim == 2 ? (B == 8 || B == 16) : (B == 4 || B == 8);
}

int launch_p2g_tile(int dim, const P2GArgs &a, int n_tiles, hipStream_t st) {
  if (dim == 2 && a.tiles.B == 8) MPM_LAUNCH((k_p2g_tile<2, 8>), n_tiles, 256, st, a);
  if (dim == 2 && a.tiles.B == 16) MPM_LAUNCH((k_p2g_tile<2, 16>), n_tiles, 256, st, a);
  if (dim == 3 && a.tiles.B == 4) MPM_LAUNCH((k_p2g_tile<3, 4>), n_tiles, 256, st, a);
  if (dim == 3 && a.tiles.B == 8) MPM_LAUNCH((k_p2g_tile<3, 8>), n_tiles, 256, st, a);
  return -1;
}

int launch_adj_scatter_tile(int dim, const AdjScatterArgs &a, int n_tiles,
                            hipStream_t st) {
  if (dim == 2 && a.tiles.B == 8) MPM_LAUNCH((k_adj_scatter_tile<2, 8>), n_tiles, 256, st, a);
  if (dim == 2 && a.tiles.B == 16) MPM_LAUNCH((k_adj_scatter_tile<2, 16>), n_tiles, 256, st, a);
  if (dim == 3 && a.tiles.B == 4) MPM_LAUNCH((k_adj_scatter_tile<3, 4>), n_tiles, 256, st, a);
  if (dim == 3 && a.tiles.B == 8) MPM_LAUNCH((k_adj_scatter_tile<3, 8>), n_tiles, 256, st, a);
  return -1;
}

int launch_p2g_sorted(int dim, const P2GArgs &a, int n_tiles, hipStream_t st) {
  if (a.mat) {
    if (a.det) {
      if (dim == 2) MPM_LAUNCH((k_p2g_sorted_pm<2, true>), n_tiles, 256, st, a);
      MPM_LAUNCH((k_p2g_sorted_pm<3, true>), n_tiles, 256, st, a);
    }
    if (dim == 2) MPM_LAUNCH((k_p2g_sorted_pm<2, false>), n_tiles, 256, st, a);
    MPM_LAUNCH((k_p2g_sorted_pm<3, false>), n_tiles, 256, st, a);
  }
  if (a.det) {
    if (dim == 2) MPM_LAUNCH((k_p2g_sorted<2, true>), n_tiles, 256, st, a);
    MPM_LAUNCH((k_p2g_sorted<3, true>), n_tiles, 256, st, a);
  }
  if (dim == 2) MPM_LAUNCH((k_p2g_sorted<2, false>), n_tiles, 256, st, a);
  MPM_LAUNCH((k_p2g_sorted<3, false>), n_tiles, 256, st, a);
}

int launch_adj_scatter_sorted(int dim, const AdjScatterArgs &a, int n_tiles,
                              hipStream_t st) {
  if (a.det) {
    if (dim == 2) MPM_LAUNCH((k_adj_scatter_sorted<2, true>), n_tiles, 256, st, a);
    MPM_LAUNCH((k_adj_scatter_sorted<3, true>), n_tiles, 256, st, a);
  }
  if (dim == 2) MPM_LAUNCH((k_adj_scatter_sorted<2, false>), n_tiles, 256, st, a);
  MPM_LAUNCH((k_adj_scatter_sorted<3, false>), n_tiles, 256, st, a);
}

int launch_p2g_cell(int dim, const P2GArgs &a, const int *cell_cnt,
                    int n_tiles, hipStream_t st) {
  const int g = (n_tiles + 3) / 4;
  if (dim == 2) MPM_LAUNCH(k_p2g_cell<2>, g, 256, st, a, cell_cnt, n_tiles);
  MPM_LAUNCH(k_p2g_cell<3>, g, 256, st, a, cell_cnt, n_tiles);
}

int launch_adj_scatter_cell(int dim, const AdjScatterArgs &a,
                            const int *cell_cnt, int n_tiles, hipStream_t st) {
  const int g = (n_tiles + 3) / 4;
  if (dim == 2) MPM_LAUNCH(k_adj_scatter_cell<2>, g, 256, st, a, cell_cnt, n_tiles);
  MPM_LAUNCH(k_adj_scatter_cell<3>, g, 256, st, a, cell_cnt, n_tiles);
}

// Persistent launches of the node-tile kernels: eight one-wave workgroups
// per CU (256 CUs), each looping over its XCD's share of the node tiles.
constexpr int PERSIST_WG = 8 * 256;

int launch_grid_nt(int dim, const GridArgs &a, hipStream_t st) {
  const int pg = std::min(a.n_nt, PERSIST_WG);
  if (a.persist) {
    if (dim == 2) MPM_LAUNCH((k_grid_nt<2, true>), pg, 64, st, a);
    MPM_LAUNCH((k_grid_nt<3, true>), pg, 64, st, a);
  }
  if (dim == 2) MPM_LAUNCH((k_grid_nt<2, false>), a.n_nt, 64, st, a);
  MPM_LAUNCH((k_grid_nt<3, false>), a.n_nt, 64, st, a);
}

int launch_adj_grid_nt(int dim, const AdjGridArgs &a, hipStream_t st) {
  const int pg = std::min(a.n_nt, PERSIST_WG);
  if (a.persist) {
    if (dim == 2) MPM_LAUNCH((k_adj_grid_nt<2, true>), pg, 64, st, a);
    MPM_LAUNCH((k_adj_grid_nt<3, true>), pg, 64, st, a);
  }
  if (dim == 2) MPM_LAUNCH((k_adj_grid_nt<2, false>), a.n_nt, 64, st, a);
  MPM_LAUNCH((k_adj_grid_nt<3, false>), a.n_nt, 64, st, a);
}

int launch_grid(int dim, const GridArgs &a, hipStream_t st) {
  if (dim == 2) MPM_LAUNCH(k_grid<2>, a.n_blocks, 256, st, a);
  MPM_LAUNCH(k_grid<3>, a.n_blocks, 256, st, a);
}

int launch_g2p_p2g_sorted(int dim, const G2P2GArgs &a, int n_tiles, hipStream_t st) {
  if (dim != 3) return -1;  // the caller only fuses 3D passes
  if (a.det) {
    if (a.mat) MPM_LAUNCH((k_g2p_p2g_sorted<3, true, true>), n_tiles, 256, st, a);
    MPM_LAUNCH((k_g2p_p2g_sorted<3, false, true>), n_tiles, 256, st, a);
  }
  if (a.mat) MPM_LAUNCH((k_g2p_p2g_sorted<3, true, false>), n_tiles, 256, st, a);
  MPM_LAUNCH((k_g2p_p2g_sorted<3, false, false>), n_tiles, 256, st, a);
}

int launch_g2p(int dim, const G2PArgs &a, hipStream_t st) {
  if (a.ctl_partial) {
    if (a.ctl_nzs > CTL_MAX_NZS || a.ctl_rows < a.n_chunks) return -1;
    if (dim == 2) MPM_LAUNCH((k_g2p<2, true>), a.n_chunks, CH, st, a);
    MPM_LAUNCH((k_g2p<3, true>), a.n_chunks, CH, st, a);
  }
  if (dim == 2) MPM_LAUNCH((k_g2p<2, false>), a.n_chunks, CH, st, a);
  MPM_LAUNCH((k_g2p<3, false>), a.n_chunks, CH, st, a);
}

int launch_adj_scatter(int dim, const AdjScatterArgs &a, hipStream_t st) {
  if (dim == 2) MPM_LAUNCH(k_adj_scatter<2>, a.n_chunks, CH, st, a);
  MPM_LAUNCH(k_adj_scatter<3>, a.n_chunks, CH, st, a);
}

int launch_adj_grid(int dim, const AdjGridArgs &a, hipStream_t st) {
  if (dim == 2) MPM_LAUNCH(k_adj_grid<2>, a.n_blocks, 256, st, a);
  MPM_LAUNCH(k_adj_grid<3>, a.n_blocks, 256, st, a);
}

// Deterministic per-actuator sum of one substep's dL/ds (deterministic
// mode): workgroup b takes actuator b, walks its scene's particles (tape
// order, a contiguous range) in a fixed strided order in FP64 and reduces
// the 256 partial sums with a fixed tree; gact[b] += the total.
__global__ __launch_bounds__(256) void k_sbar_reduce(const DevScene *scenes,
                                                     const int *act_scene,
                                                     const int *tile_start,
                                                     const int *act_id,
                                                     const float *sb_part,
                                                     int dim, double *gact) {
  __shared__ double s[256];
  const int b = blockIdx.x, t = threadIdx.x;
  const DevScene sc = scenes[act_scene[b]];
  const int a = b - sc.act_off;
  const int nts = sc.nt * sc.nt * (dim == 3 ? sc.nt : 1);
  const int p0 = tile_start[sc.tile_off], p1 = tile_start[sc.tile_off + nts];
  double acc = 0.0;
  for (int p = p0 + t; p < p1; p += 256)
    if (act_id[p] == a) acc += (double)sb_part[p];
  s[t] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) s[t] += s[t + h];
    __syncthreads();
  }
  if (t == 0) gact[b] += s[0];
}

int launch_sbar_reduce(const DevScene *scenes, const int *act_scene, int n_act,
                       const int *tile_start, const int *act_id, const float *sb_part,
                       int dim, double *gact, hipStream_t st) {
  MPM_LAUNCH(k_sbar_reduce, n_act, 256, st, scenes, act_scene, tile_start, act_id,
             sb_part, dim, gact);
}

// Deterministic ranks in a cell at binning: each cell's particles (listed
// at their atomic rank) are sorted by index, one thread per cell, and the
// rank becomes the position in that order.
__global__ __launch_bounds__(256) void k_cell_fill(const int *ptile, const int *pcell,
                                                   const int *prank, const int *cell_start,
                                                   int cpt, int N, int *list) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= N) return;
  const int tile = ptile[p];
  if (tile < 0) return;
  list[cell_start[(int64_t)tile * cpt + pcell[p]] + prank[p]] = p;
}

__global__ __launch_bounds__(256) void k_cell_sort(const int *cell_start, int n_cells,
                                                   int *list, int *prank) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= n_cells) return;
  const int lo = cell_start[c], hi = cell_start[c + 1];
  for (int i = lo + 1; i < hi; ++i) {
    const int v = list[i];
    int k = i - 1;
    while (k >= lo && list[k] > v) {
      list[k + 1] = list[k];
      --k;
    }
    list[k + 1] = v;
  }
  for (int i = lo; i < hi; ++i) prank[list[i]] = i - lo;
}

int launch_cell_fill(const int *ptile, const int *pcell, const int *prank,
                     const int *cell_start, int cpt, int N, int *list, hipStream_t st) {
  MPM_LAUNCH(k_cell_fill, blocks_for(N), 256, st, ptile, pcell, prank, cell_start, cpt,
             N, list);
}

int launch_cell_sort(const int *cell_start, int n_cells, int *list, int *prank,
                     hipStream_t st) {
  MPM_LAUNCH(k_cell_sort, blocks_for(n_cells), 256, st, cell_start, n_cells, list, prank);
}

int launch_adj_gather_scatter(int dim, const AdjFusedArgs &a, int n_tiles, hipStream_t st) {
  if (dim != 3) return -1;  // the caller only fuses 3D passes
  if (a.det) MPM_LAUNCH((k_adj_gather_scatter<3, true>), n_tiles, 256, st, a);
  MPM_LAUNCH((k_adj_gather_scatter<3, false>), n_tiles, 256, st, a);
}

int launch_adj_gather(int dim, const AdjGatherArgs &a, hipStream_t st) {
  if (a.mat) {
    if (dim == 2) MPM_LAUNCH((k_adj_gather<2, true>), a.n_chunks, CH, st, a);
    MPM_LAUNCH((k_adj_gather<3, true>), a.n_chunks, CH, st, a);
  }
  if (dim == 2) MPM_LAUNCH((k_adj_gather<2, false>), a.n_chunks, CH, st, a);
  MPM_LAUNCH((k_adj_gather<3, false>), a.n_chunks, CH, st, a);
}

// Per-particle material field [3][N] (mu, la, m_p) from E_p and rho_p
// (nullable: the scene's E or rho), caller order.
__global__ __launch_bounds__(256) void k_mat_field(const DevScene *scenes,
                                                   const int *pscene, int N,
                                                   const float *E_p,
                                                   const float *rho_p, float *mat) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= N) return;
  const DevScene sc = scenes[pscene[p]];
  float mu = sc.mu, la = sc.la;
  if (E_p) {
    const float E = E_p[p];
    mu = E / (2.0f * (1.0f + sc.nu));
    la = E * sc.nu / ((1.0f + sc.nu) * (1.0f - 2.0f * sc.nu));
  }
  mat[p] = mu;
  mat[N + p] = la;
  mat[2 * N + p] = rho_p ? rho_p[p] * sc.V0 : sc.mp;
}

// dL/dE_p, dL/drho_p (caller order) from the accumulated dL/dmu, dL/dla,
// dL/dm_p [3][N] of the reverse pass (tape order; perm: tape -> caller,
// null when the tape is in caller order).
__global__ __launch_bounds__(256) void k_mat_grad(const DevScene *scenes,
                                                  const int *pscene, int N,
                                                  const int *perm, const float *gmat,
                                                  float *g_E, float *g_rho) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const int p = perm ? perm[i] : i;
  if (p < 0 || p >= N) return;
  const DevScene sc = scenes[pscene[p]];
  const float dmu = 1.0f / (2.0f * (1.0f + sc.nu));
  const float dla = sc.nu / ((1.0f + sc.nu) * (1.0f - 2.0f * sc.nu));
  if (g_E) g_E[p] = gmat[i] * dmu + gmat[N + i] * dla;
  if (g_rho) g_rho[p] = gmat[2 * N + i] * sc.V0;
}

// Descriptors and cleared grid of the allocation-free single substep, all
// from kernel arguments (a captured graph replays them): the scene, its
// chunks of CH particles and node blocks of 256 nodes, a copy of the
// actuator ids in which an id outside [-1, n_act) becomes passive and sets
// EB_ACT_ID, and m = p = 0 on the scene's nodes.
__global__ __launch_bounds__(256) void k_noalloc_setup(NoAllocArgs a) {
  const int64_t n = (int64_t)gridDim.x * 256;
  const int64_t t0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int nch = (a.N + CH - 1) / CH, nb = (int)((a.nodes + 255) / 256);
  if (t0 == 0) *a.scene = a.sc;
  for (int64_t i = t0; i < nch; i += n)
    a.chunks[i] = Chunk{0, (int)(i * CH), (int)min<int64_t>(CH, a.N - i * CH), 0};
  for (int64_t i = t0; i < nb; i += n)
    a.blocks[i] = GridBlock{0, (int)(i * 256), (int)min<int64_t>(256, a.nodes - i * 256), 0};
  unsigned eb = 0;
  for (int64_t i = t0; i < a.N; i += n) {
    int j = a.act_id_in ? a.act_id_in[i] : -1;
    if (j < -1 || j >= a.sc.n_act) {
      eb |= EB_ACT_ID;
      j = -1;
    }
    a.act_id[i] = j;
  }
  if (eb) atomicOr(a.err, eb);
  for (int64_t i = t0; i < (int64_t)(1 + a.dim) * a.nodes; i += n) {
    if (i < a.nodes) a.gm[i] = 0.0f;
    else a.gp[((i - a.nodes) / a.nodes) * a.G + (i - a.nodes) % a.nodes] = 0.0f;
  }
}

int launch_noalloc_setup(const NoAllocArgs &a, hipStream_t st) {
  const int64_t work = std::max<int64_t>(a.N, (1 + a.dim) * a.nodes);
  const int g = (int)std::min<int64_t>(std::max<int64_t>(blocks_for(work), 1), 2048);
  MPM_LAUNCH(k_noalloc_setup, g, 256, st, a);
}

int launch_fill_f32(float *p, int64_t n, hipStream_t st) {
  const int g = (int)std::min<int64_t>(blocks_for(n), 4096);
  MPM_LAUNCH(k_fill<float>, g, 256, st, p, n);
}

int launch_fill_f64(double *p, int64_t n, hipStream_t st) {
  const int g = (int)std::min<int64_t>(blocks_for(n), 4096);
  MPM_LAUNCH(k_fill<double>, g, 256, st, p, n);
}

int launch_fill_i32(int *p, int64_t n, hipStream_t st) {
  const int g = (int)std::min<int64_t>(blocks_for(n), 4096);
  MPM_LAUNCH(k_fill<int>, g, 256, st, p, n);
}

int launch_sort_count(int dim, const SortArgs &a, hipStream_t st) {
  if (dim == 2) MPM_LAUNCH(k_sort_count<2>, blocks_for(a.N), 256, st, a);
  MPM_LAUNCH(k_sort_count<3>, blocks_for(a.N), 256, st, a);
}

int launch_scan_i32(const int *in, int *out, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_i32, dim3(1), dim3(1024), 0, st, in, out, n);
  return hip_rc(hipGetLastError());
}

int launch_sort_place(int dim, const SortArgs &a, const int *tile_start,
                      int *perm, hipStream_t st) {
  if (dim == 2)
    MPM_LAUNCH(k_sort_place<2>, blocks_for(a.N), 256, st, a, tile_start, perm);
  MPM_LAUNCH(k_sort_place<3>, blocks_for(a.N), 256, st, a, tile_start, perm);
}

int launch_chunk_count(const int *tile_cnt, int n, int *nch, hipStream_t st) {
  MPM_LAUNCH(k_chunk_count, blocks_for(n), 256, st, tile_cnt, n, nch);
}

int launch_nonempty_flag(const int *tile_cnt, int n, int *flag, hipStream_t st) {
  MPM_LAUNCH(k_nonempty_flag, blocks_for(n), 256, st, tile_cnt, n, flag);
}

int launch_nt_cand(const DevScene *scenes, const int *nt_scene, int n_nt,
                   const int *tile_cnt, int *cand, hipStream_t st) {
  MPM_LAUNCH(k_nt_cand, (n_nt + 255) / 256, 256, st, scenes, nt_scene, n_nt, tile_cnt, cand);
}

int launch_compact(const int *flag, const int *pos, int n, int *list,
                   hipStream_t st) {
  MPM_LAUNCH(k_compact, blocks_for(n), 256, st, flag, pos, n, list);
}

int launch_build_chunks(const int *tile_cnt, const int *tile_start,
                        const int *chunk_start, const int *tile_scene, int n,
                        Chunk *chunks, hipStream_t st) {
  MPM_LAUNCH(k_build_chunks, blocks_for(n), 256, st, tile_cnt, tile_start,
             chunk_start, tile_scene, n, chunks);
}

int launch_permute_rows(const float *in, float *out, const int *perm, int N,
                        int ld, int ncomp, int scatter, hipStream_t st) {
  MPM_LAUNCH(k_permute_rows, blocks_for(N), 256, st, in, out, perm, N, ld,
             ncomp, scatter);
}

int launch_permute_i32(const int *in, int *out, const int *perm, int N,
                       hipStream_t st) {
  MPM_LAUNCH(k_permute_i32, blocks_for(N), 256, st, in, out, perm, N);
}

int launch_ctl_forward(const CtlArgs &a, hipStream_t st) {
  const int nzs = 2 * a.dim * a.n_comp;
  if (a.N < 1 || nzs == 0 || nzs > CTL_MAX_NZS || a.n_act > 64) return -1;
  const int rows = ctl_rows(a.N);
  if (a.dim == 2)
    hipLaunchKernelGGL(k_ctl_partial<2>, dim3(rows), dim3(256), 0, st, a, rows);
  else if (a.dim == 3)
    hipLaunchKernelGGL(k_ctl_partial<3>, dim3(rows), dim3(256), 0, st, a, rows);
  else
    return -1;
  const int rc = hip_rc(hipGetLastError());
  if (rc) return rc;
  MPM_LAUNCH(k_ctl_reduce, nzs, 256, st, a, rows);
}

int ctl_rows(int N) { return std::min((N + 255) / 256, 2048); }

int launch_ctl_reduce(const CtlArgs &a, int n_rows, hipStream_t st) {
  const int nzs = 2 * a.dim * a.n_comp;
  if (n_rows < 1 || nzs == 0 || nzs > CTL_MAX_NZS || a.n_act > 64) return -1;
  MPM_LAUNCH(k_ctl_reduce, nzs, 256, st, a, n_rows);
}

int launch_ctl_adjoint(const CtlAdjArgs &a, hipStream_t st) {
  if (a.N < 1 || a.n_act > 64 || 2 * a.dim * a.n_comp > CTL_MAX_NZS) return -1;
  const int n_wg = std::min((a.N + 255) / 256, CTL_WG);
  MPM_LAUNCH(k_ctl_adjoint, n_wg, 256, st, a, n_wg);
}

int launch_gact_store(const double *src, float *dst, int64_t n, int accumulate,
                      hipStream_t st) {
  MPM_LAUNCH(k_gact_store, blocks_for(n), 256, st, src, dst, n, accumulate);
}

int launch_act_bank_fwd(int T, int n_act, int n_freq, float dt,
                        const float *freq, const float *amp,
                        const float *phase, float *act, hipStream_t st) {
  MPM_LAUNCH(k_act_bank_fwd, blocks_for((int64_t)T * n_act), 256, st, T, n_act,
             n_freq, dt, freq, amp, phase, act);
}

int launch_act_bank_bwd(int T, int n_act, int n_freq, float dt,
                        const float *freq, const float *amp,
                        const float *phase, const float *g_act, float *g_amp,
                        float *g_phase, hipStream_t st) {
  MPM_LAUNCH(k_act_bank_bwd, n_act * n_freq, 256, st, T, n_act, n_freq, dt,
             freq, amp, phase, g_act, g_amp, g_phase);
}

}  // namespace mpm

namespace mpm {
int launch_mat_field(const DevScene *scenes, const int *pscene, int N,
                     const float *E_p, const float *rho_p, float *mat, hipStream_t st) {
  MPM_LAUNCH(k_mat_field, (N + 255) / 256, 256, st, scenes, pscene, N, E_p, rho_p, mat);
}
int launch_mat_grad(const DevScene *scenes, const int *pscene, int N, const int *perm,
                    const float *gmat, float *g_E, float *g_rho, hipStream_t st) {
  MPM_LAUNCH(k_mat_grad, (N + 255) / 256, 256, st, scenes, pscene, N, perm, gmat, g_E, g_rho);
}
}  // namespace mpm
