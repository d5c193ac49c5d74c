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

// Returns false (and sets eb) when det F <= 0 or is not finite.
template <int D>
__device__ __forceinline__ bool stress(const DevScene &sc, const float *F,
                                       float s_act, bool has_act, Stress<D> &S,
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
      S.Pt[k] = sc.mu * (F[k] - S.FiT[k]) + sc.la * S.lnJ * S.FiT[k] +
                F[k] * S.sigma[b];
    }
  return true;
}

// G = kG P_t F^T + m_p C with kG = -(4/dx^2) dt V0.
template <int D>
__device__ __forceinline__ void affine_G(const DevScene &sc, const float *Pt,
                                         const float *F, const float *C,
                                         float *G) {
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      float s = 0.0f;
#pragma unroll
      for (int g = 0; g < D; ++g) s += Pt[a * D + g] * F[b * D + g];
      G[a * D + b] = sc.kG * s + sc.mp * C[a * D + b];
    }
}

__device__ __forceinline__ int chunk_id() { return blockIdx.x; }

// ---------------------------------------------------------------------------
// step 1: P2G scatter
// ---------------------------------------------------------------------------

template <int D>
__global__ __launch_bounds__(CH) void k_p2g(P2GArgs A) {
  __shared__ float s_grid[(D + 1) * LDS_NODES];
  const Chunk ch = A.chunks[chunk_id()];
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

  float G[D * D], mv[D];
  if (ok) {
    float F[D * D], C[D * D], v[D];
    load_mat<D>(A.s.F, A.ld, p, F);
    load_mat<D>(A.s.C, A.ld, p, C);
    load_vec<D>(A.s.v, A.ld, p, v);
    const int j = A.act_id[p];
    const float s_act = j >= 0 ? A.act[sc.act_off + j] : 0.0f;
    Stress<D> S;
    ok = stress<D>(sc, F, s_act, j >= 0, S, eb);
    if (ok) {
      affine_G<D>(sc, S.Pt, F, C, G);
#pragma unroll
      for (int a = 0; a < D; ++a) mv[a] = sc.mp * v[a];
    }
  }
  if (box.lds) {
    for (int i = t; i < (D + 1) * LDS_NODES; i += CH) s_grid[i] = 0.0f;
    __syncthreads();
  }
  if (ok) {
    float w[D][3];
#pragma unroll
    for (int a = 0; a < D; ++a) bspline_w(f[a], w[a]);
    // m_p v_p + G (x_i - x_p) is affine in the offset o: c0 + sum_b o_b Gb_b
    float c0[D], Gdx[D][D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      float s = mv[a];
#pragma unroll
      for (int b = 0; b < D; ++b) {
        Gdx[a][b] = G[a * D + b] * sc.dx;
        s -= Gdx[a][b] * f[b];
      }
      c0[a] = s;
    }
    const int lbase = box.lds ? box_index<D>(box, base) : 0;
    const int gbase = sc.g_off + node_index<D>(base, sc.n);
    if constexpr (D == 2) {
#pragma unroll
      for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
        for (int o1 = 0; o1 < 3; ++o1) {
          const float N = w[0][o0] * w[1][o1];
          float val[2];
#pragma unroll
          for (int a = 0; a < 2; ++a)
            val[a] = N * (c0[a] + Gdx[a][0] * o0 + Gdx[a][1] * o1);
          if (box.lds) {
            const int li = lbase + o0 * box.e[1] + o1;
            lds_add(&s_grid[li], N * sc.mp);
            lds_add(&s_grid[LDS_NODES + li], val[0]);
            lds_add(&s_grid[2 * LDS_NODES + li], val[1]);
          } else {
            const int64_t gi = gbase + o0 * sc.n + o1;
            gmem_add(&A.gm[gi], N * sc.mp);
            gmem_add(&A.gp[gi], val[0]);
            gmem_add(&A.gp[A.G + gi], val[1]);
          }
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
            float val[3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
              val[a] = N * (c0[a] + Gdx[a][0] * o0 + Gdx[a][1] * o1 +
                            Gdx[a][2] * o2);
            if (box.lds) {
              const int li = lbase + (o0 * box.e[1] + o1) * box.e[2] + o2;
              lds_add(&s_grid[li], N * sc.mp);
              lds_add(&s_grid[LDS_NODES + li], val[0]);
              lds_add(&s_grid[2 * LDS_NODES + li], val[1]);
              lds_add(&s_grid[3 * LDS_NODES + li], val[2]);
            } else {
              const int64_t gi = gbase + (o0 * sc.n + o1) * sc.n + o2;
              gmem_add(&A.gm[gi], N * sc.mp);
              gmem_add(&A.gp[gi], val[0]);
              gmem_add(&A.gp[A.G + gi], val[1]);
              gmem_add(&A.gp[2 * A.G + gi], val[2]);
            }
          }
        }
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

template <int D>
__global__ __launch_bounds__(256) void k_grid(GridArgs A) {
  const GridBlock gb = A.blocks[blockIdx.x];
  if ((int)threadIdx.x >= gb.count) return;
  const DevScene sc = A.scenes[gb.scene];
  const int li = gb.start + threadIdx.x;
  const int64_t gi = sc.g_off + li;
  const float m = A.gm[gi];
  const bool wall = is_wall<D>(li, sc.n, sc.wall);
  float v[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float va = 0.0f;
    if (m > 0.0f) va = A.gp[a * A.G + gi] / m + sc.dt * sc.g[a];
    v[a] = wall ? 0.0f : va;
  }
#pragma unroll
  for (int a = 0; a < D; ++a) A.gv[a * A.G + gi] = v[a];
  if (A.zero_mp && m != 0.0f) {
    A.gm[gi] = 0.0f;
#pragma unroll
    for (int a = 0; a < D; ++a) A.gp[a * A.G + gi] = 0.0f;
  }
}

// ---------------------------------------------------------------------------
// step 3: G2P gather + F/C/x update
// ---------------------------------------------------------------------------

template <int D>
__global__ __launch_bounds__(CH) void k_g2p(G2PArgs A) {
  __shared__ float s_v[D * LDS_NODES];
  const Chunk ch = A.chunks[chunk_id()];
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
  if (box.lds) {
    for (int i = t; i < box.vol; i += CH) {
      const int64_t gi = sc.g_off + box_node<D>(box, i, sc.n);
#pragma unroll
      for (int a = 0; a < D; ++a) s_v[a * LDS_NODES + i] = A.gv[a * A.G + gi];
    }
    __syncthreads();
  }
  if (!active) return;
  float F[D * D];
  load_mat<D>(A.s.F, A.ld, p, F);
  if (!ok) {
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
          const int64_t gi = gbase + o0 * sc.n + o1;
          vi[0] = A.gv[gi];
          vi[1] = A.gv[A.G + gi];
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
#pragma unroll
    for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
      for (int o1 = 0; o1 < 3; ++o1) {
        const float w01 = w[0][o0] * w[1][o1];
#pragma unroll
        for (int o2 = 0; o2 < 3; ++o2) {
          const float N = w01 * w[2][o2];
          const float d0 = (float)o0 - f[0], d1 = (float)o1 - f[1],
                      d2 = (float)o2 - f[2];
          float vi[3];
          if (box.lds) {
            const int li = lbase + (o0 * box.e[1] + o1) * box.e[2] + o2;
            vi[0] = s_v[li];
            vi[1] = s_v[LDS_NODES + li];
            vi[2] = s_v[2 * LDS_NODES + li];
          } else {
            const int64_t gi = gbase + (o0 * sc.n + o1) * sc.n + o2;
            vi[0] = A.gv[gi];
            vi[1] = A.gv[A.G + gi];
            vi[2] = A.gv[2 * A.G + gi];
          }
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const float Nv = N * vi[a];
            vn[a] += Nv;
            B[a * 3 + 0] += Nv * d0;
            B[a * 3 + 1] += Nv * d1;
            B[a * 3 + 2] += Nv * d2;
          }
        }
      }
  }
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
}

// ---------------------------------------------------------------------------
// reverse R1: adjoint of G2P, a particle -> grid scatter (supplement A-C)
// ---------------------------------------------------------------------------

template <int D>
__global__ __launch_bounds__(CH) void k_adj_scatter(AdjScatterArgs A) {
  __shared__ float s_grid[D * LDS_NODES];
  const Chunk ch = A.chunks[chunk_id()];
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
  float vt[D], Ct[D * D];
  if (ok) {
    float F[D * D], gx[D], gv[D], gC[D * D], gF[D * D];
    load_mat<D>(A.s.F, A.ld, p, F);
    load_vec<D>(A.g1.x, A.ld, p, gx);
    load_vec<D>(A.g1.v, A.ld, p, gv);
    load_mat<D>(A.g1.C, A.ld, p, gC);
    load_mat<D>(A.g1.F, A.ld, p, gF);
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
  }
  if (box.lds) {
    for (int i = t; i < D * LDS_NODES; i += CH) s_grid[i] = 0.0f;
    __syncthreads();
  }
  if (ok) {
    float w[D][3];
#pragma unroll
    for (int a = 0; a < D; ++a) bspline_w(f[a], w[a]);
    // (C): vt + (4/dx^2) Ct (x_i - x_p) is affine in o
    float c0[D], Cdx[D][D];
    const float cs = sc.Dinv * sc.dx;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      float s = vt[a];
#pragma unroll
      for (int b = 0; b < D; ++b) {
        Cdx[a][b] = cs * Ct[a * D + b];
        s -= Cdx[a][b] * f[b];
      }
      c0[a] = s;
    }
    const int lbase = box.lds ? box_index<D>(box, base) : 0;
    const int gbase = sc.g_off + node_index<D>(base, sc.n);
    if constexpr (D == 2) {
#pragma unroll
      for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
        for (int o1 = 0; o1 < 3; ++o1) {
          const float N = w[0][o0] * w[1][o1];
          float val[2];
#pragma unroll
          for (int a = 0; a < 2; ++a)
            val[a] = N * (c0[a] + Cdx[a][0] * o0 + Cdx[a][1] * o1);
          if (box.lds) {
            const int li = lbase + o0 * box.e[1] + o1;
            lds_add(&s_grid[li], val[0]);
            lds_add(&s_grid[LDS_NODES + li], val[1]);
          } else {
            const int64_t gi = gbase + o0 * sc.n + o1;
            gmem_add(&A.vbar[gi], val[0]);
            gmem_add(&A.vbar[A.G + gi], val[1]);
          }
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
            float val[3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
              val[a] = N * (c0[a] + Cdx[a][0] * o0 + Cdx[a][1] * o1 +
                            Cdx[a][2] * o2);
            if (box.lds) {
              const int li = lbase + (o0 * box.e[1] + o1) * box.e[2] + o2;
              lds_add(&s_grid[li], val[0]);
              lds_add(&s_grid[LDS_NODES + li], val[1]);
              lds_add(&s_grid[2 * LDS_NODES + li], val[2]);
            } else {
              const int64_t gi = gbase + (o0 * sc.n + o1) * sc.n + o2;
              gmem_add(&A.vbar[gi], val[0]);
              gmem_add(&A.vbar[A.G + gi], val[1]);
              gmem_add(&A.vbar[2 * A.G + gi], val[2]);
            }
          }
        }
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

// ---------------------------------------------------------------------------
// reverse R2: adjoint of the grid operations (supplement D-E)
// ---------------------------------------------------------------------------

template <int D>
__global__ __launch_bounds__(256) void k_adj_grid(AdjGridArgs A) {
  const GridBlock gb = A.blocks[blockIdx.x];
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
  float mb = 0.0f;
  if (m > 0.0f) {
    const float im = 1.0f / m;
    float dot = 0.0f;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const float vhat = A.gp[a * A.G + gi] / m;  // before gravity (E)
      v[a] = wall ? 0.0f : vhat + sc.dt * sc.g[a];
      pb[a] = wall ? 0.0f : vb[a] * im;          // (D)
      dot += vhat * vb[a];
    }
    mb = wall ? 0.0f : -dot * im;                // (E)
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

// ---------------------------------------------------------------------------
// reverse R3: adjoint of P2G and of the particle update, a grid -> particle
// gather (supplement F-K)
// ---------------------------------------------------------------------------

template <int D>
__global__ __launch_bounds__(CH) void k_adj_gather(AdjGatherArgs A) {
  constexpr int NCH = 2 * D + 1;  // staged channels: pbar[D], mbar, v[D]
  __shared__ float s_n[NCH * LDS_NODES];
  __shared__ double s_act[LDS_ACT];
  const Chunk ch = A.chunks[chunk_id()];
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
  const bool act_lds = sc.n_act <= LDS_ACT && A.gact != nullptr;
  if (act_lds)
    for (int i = t; i < sc.n_act; i += CH) s_act[i] = 0.0;
  if (box.lds) {
    for (int i = t; i < box.vol; i += CH) {
      const int64_t gi = sc.g_off + box_node<D>(box, i, sc.n);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        s_n[a * LDS_NODES + i] = A.pbar[a * A.G + gi];
        s_n[(D + 1 + a) * LDS_NODES + i] = A.gv[a * A.G + gi];
      }
      s_n[D * LDS_NODES + i] = A.mbar[gi];
    }
  }
  __syncthreads();

  float sb_act = 0.0f;
  int j_act = -1;
  if (ok) {
    float v[D], C[D * D], F[D * D];
    load_vec<D>(A.s.v, A.ld, p, v);
    load_mat<D>(A.s.C, A.ld, p, C);
    load_mat<D>(A.s.F, A.ld, p, F);
    j_act = A.act_id[p];
    const float s_act = j_act >= 0 ? A.act[sc.act_off + j_act] : 0.0f;
    Stress<D> S;
    ok = stress<D>(sc, F, s_act, j_act >= 0, S, eb);
    if (ok) {
      float G[D * D];
      affine_G<D>(sc, S.Pt, F, C, G);
      float gx1[D], gv1[D], gC1[D * D], gF1[D * D];
      load_vec<D>(A.g1.x, A.ld, p, gx1);
      load_vec<D>(A.g1.v, A.ld, p, gv1);
      load_mat<D>(A.g1.C, A.ld, p, gC1);
      load_mat<D>(A.g1.F, A.ld, p, gF1);
      float vt[D], Ct[D * D];
#pragma unroll
      for (int a = 0; a < D; ++a) vt[a] = gv1[a] + sc.dt * gx1[a];  // (A)
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {  // (B)
          float s = 0.0f;
#pragma unroll
          for (int g = 0; g < D; ++g) s += gF1[a * D + g] * F[b * D + g];
          Ct[a * D + b] = gC1[a * D + b] + sc.dt * s;
        }
      float w[D][3], dw[D][3];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        bspline_w(f[a], w[a]);
        bspline_dw(f[a], sc.inv_dx, dw[a]);
      }
      // affine-in-o pieces:  Ct (x_i - x_p) and m v + G (x_i - x_p)
      float cC[D], Cdx[D][D], cq[D], Gdx[D][D];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        float s1 = 0.0f, s2 = sc.mp * v[a];
#pragma unroll
        for (int b = 0; b < D; ++b) {
          Cdx[a][b] = Ct[a * D + b] * sc.dx;
          Gdx[a][b] = G[a * D + b] * sc.dx;
          s1 -= Cdx[a][b] * f[b];
          s2 -= Gdx[a][b] * f[b];
        }
        cC[a] = s1;
        cq[a] = s2;
      }
      float xb[D], Spb[D] = {}, Sv[D] = {}, Gb[D * D] = {};
#pragma unroll
      for (int a = 0; a < D; ++a) xb[a] = gx1[a];  // (J) direct term
      const int lbase = box.lds ? box_index<D>(box, base) : 0;
      const int gbase = sc.g_off + node_index<D>(base, sc.n);

      auto node = [&](int li, int64_t gi, float N, const float *gN,
                      const float *dl) {
        float pb[D], vi[D], mb;
        if (box.lds) {
#pragma unroll
          for (int a = 0; a < D; ++a) {
            pb[a] = s_n[a * LDS_NODES + li];
            vi[a] = s_n[(D + 1 + a) * LDS_NODES + li];
          }
          mb = s_n[D * LDS_NODES + li];
        } else {
#pragma unroll
          for (int a = 0; a < D; ++a) {
            pb[a] = A.pbar[a * A.G + gi];
            vi[a] = A.gv[a * A.G + gi];
          }
          mb = A.mbar[gi];
        }
        float s_all = sc.mp * mb;  // (J) m-term
#pragma unroll
        for (int a = 0; a < D; ++a) {
          float Cd = cC[a], q = cq[a];
#pragma unroll
          for (int b = 0; b < D; ++b) {
            Cd += Cdx[a][b] * dl[b];
            q += Gdx[a][b] * dl[b];
          }
          // (J) v-term, C-term (N part), p-term (N part)
          s_all += vt[a] * vi[a] + sc.Dinv * vi[a] * Cd + pb[a] * q;
          const float Npb = N * pb[a];
          Spb[a] += Npb;          // (F), and the delta-part of (J)
          Sv[a] += N * vi[a];     // delta-part of the (J) C-term
#pragma unroll
          for (int b = 0; b < D; ++b)
            Gb[a * D + b] += Npb * (dl[b] - f[b]);  // dL/dG, in units of dx
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
            const float dl[2] = {(float)o0, (float)o1};
            node(lbase + o0 * box.e[1] + o1, gbase + o0 * sc.n + o1, N, gN,
                 dl);
          }
      } else {
#pragma unroll
        for (int o0 = 0; o0 < 3; ++o0)
#pragma unroll
          for (int o1 = 0; o1 < 3; ++o1) {
            const float w01 = w[0][o0] * w[1][o1];
            const float d01 = dw[0][o0] * w[1][o1];
            const float w0d1 = w[0][o0] * dw[1][o1];
#pragma unroll
            for (int o2 = 0; o2 < 3; ++o2) {
              const float N = w01 * w[2][o2];
              const float gN[3] = {d01 * w[2][o2], w0d1 * w[2][o2],
                                   w01 * dw[2][o2]};
              const float dl[3] = {(float)o0, (float)o1, (float)o2};
              node(lbase + (o0 * box.e[1] + o1) * box.e[2] + o2,
                   gbase + (o0 * sc.n + o1) * sc.n + o2, N, gN, dl);
            }
          }
      }
      // (J) delta-parts: -sum N [ (4/dx^2) Ct^T v_i + G^T p_i ]
#pragma unroll
      for (int c = 0; c < D; ++c) {
        float s = 0.0f;
#pragma unroll
        for (int a = 0; a < D; ++a)
          s += sc.Dinv * Ct[a * D + c] * Sv[a] + G[a * D + c] * Spb[a];
        xb[c] -= s;
      }
      float vb[D], Cb[D * D], Ptb[D * D], Fb[D * D];
#pragma unroll
      for (int a = 0; a < D; ++a) vb[a] = sc.mp * Spb[a];  // (F)
#pragma unroll
      for (int k = 0; k < D * D; ++k) {
        Gb[k] *= sc.dx;            // dL/dG = sum N p_i (x_i - x_p)^T
        Cb[k] = sc.mp * Gb[k];     // (I)
      }
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
      // (H) dL/dF: update term (I + dt C^{n+1})^T dL/dF^{n+1}
      float C1[D * D];
      load_mat<D>(A.C1, A.ld, p, C1);
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
      const float cmu = sc.mu - sc.la * S.lnJ;
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
          float s = 0.0f;
#pragma unroll
          for (int g = 0; g < D; ++g) s += T1[a * D + g] * S.FiT[g * D + b];
          Fb[a * D + b] +=
              sc.mu * Ptb[a * D + b] + cmu * s + sc.la * inner * S.FiT[a * D + b];
        }
      // (K) dL/dsigma_aa = (F^T dL/dP_t)_aa;  s-bar = sum_a axis_a sigma-bar_aa
      if (j_act >= 0) {
#pragma unroll
        for (int a = 0; a < D; ++a) {
          float s = 0.0f;
#pragma unroll
          for (int g = 0; g < D; ++g) s += F[g * D + a] * Ptb[g * D + a];
          sb_act += sc.axis[a] * s;
        }
      }
      if (!(finite_all(xb, D) && finite_all(vb, D) && finite_all(Cb, D * D) &&
            finite_all(Fb, D * D)))
        eb |= EB_NONFINITE;
      store_vec<D>(A.g0.x, A.ld, p, xb);
      store_vec<D>(A.g0.v, A.ld, p, vb);
      store_mat<D>(A.g0.C, A.ld, p, Cb);
      store_mat<D>(A.g0.F, A.ld, p, Fb);
    }
  }
  if (active && !ok) {
    float z[D * D] = {};
    store_vec<D>(A.g0.x, A.ld, p, z);
    store_vec<D>(A.g0.v, A.ld, p, z);
    store_mat<D>(A.g0.C, A.ld, p, z);
    store_mat<D>(A.g0.F, A.ld, p, z);
  }
  if (eb) atomicOr(A.err, eb);
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
  atomicAdd(&A.tile_cnt[tile], 1);
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
  if (i < N) out[i] = in[perm[i]];
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

int launch_grid(int dim, const GridArgs &a, hipStream_t st) {
  if (dim == 2) MPM_LAUNCH(k_grid<2>, a.n_blocks, 256, st, a);
  MPM_LAUNCH(k_grid<3>, a.n_blocks, 256, st, a);
}

int launch_g2p(int dim, const G2PArgs &a, hipStream_t st) {
  if (dim == 2) MPM_LAUNCH(k_g2p<2>, a.n_chunks, CH, st, a);
  MPM_LAUNCH(k_g2p<3>, a.n_chunks, CH, st, a);
}

int launch_adj_scatter(int dim, const AdjScatterArgs &a, hipStream_t st) {
  if (dim == 2) MPM_LAUNCH(k_adj_scatter<2>, a.n_chunks, CH, st, a);
  MPM_LAUNCH(k_adj_scatter<3>, a.n_chunks, CH, st, a);
}

int launch_adj_grid(int dim, const AdjGridArgs &a, hipStream_t st) {
  if (dim == 2) MPM_LAUNCH(k_adj_grid<2>, a.n_blocks, 256, st, a);
  MPM_LAUNCH(k_adj_grid<3>, a.n_blocks, 256, st, a);
}

int launch_adj_gather(int dim, const AdjGatherArgs &a, hipStream_t st) {
  if (dim == 2) MPM_LAUNCH(k_adj_gather<2>, a.n_chunks, CH, st, a);
  MPM_LAUNCH(k_adj_gather<3>, a.n_chunks, CH, st, a);
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
