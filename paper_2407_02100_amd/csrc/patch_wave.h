// Patch smoother kernel for 3D, constant coefficient, one patch per wavefront
// (the hot kernel of the V-cycle on the finest levels).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace vps {

// ---------------------------------------------------------------------------
// Patch smoother, 3D, constant coefficient: one patch at a time per wavefront.
//
// With the exact local solver the update of Algorithm 4,
//   u_int <- ubar_int + A_j^{-1} (b_j - Abar_j ubar),
// equals A_j^{-1} (b_j - A_{j,Gamma} ubar_Gamma), because the interior rows
// of Abar_j split into A_j (interior columns) and A_{j,Gamma} (patch boundary
// columns).  The kernel therefore evaluates the local residual of the
// closure with the interior values taken as zero, applies the fast
// diagonalisation and stores the result as the new interior.
//
// Fast diagonalisation in even/odd form: the 1D patch problem is symmetric
// under reversal of the node order, so each eigenvector is symmetric (K of
// them) or antisymmetric (K-1).  T^T v then needs the folded sums/differences
// of v and the K x K and (K-1) x (K-1) blocks Te, To only; the modes are kept
// in the internal order [symmetric..., antisymmetric...] throughout, and each
// lane forms its reciprocal eigenvalue sums 1/(lam_x + lam_y + lam_z) from
// the 1D eigenvalues in that order (kernel arguments): a table in memory
// would cost vector-memory instructions, the unit this kernel is bound by.
//
// Stages of the wave64 that owns a patch:
//   0. every global load of the patch, issued before any arithmetic so that
//      they are in flight together: the closure columns (y, x) along z
//      (boundary columns carry 2K+1 values, interior columns only their two
//      end values) and the right-hand side columns of the interior;
//   1. z contraction of the closure columns;  2. y contraction of the
//      (z-out, x) lines;  3. x contraction of the (z-out, y-out) lines, local
//      residual, T^T along x;  4. T^T along y;  5. T^T along z and 1/Lambda;
//   6. T along x;  7. T along y;  8. T along z and store, plane by plane.
// One wave64 (one workgroup) per patch.  Workgroups are mapped so that each
// of the 8 XCDs owns one contiguous slab of the color's patches
// (lexicographic order), which keeps the closure planes that neighbouring
// patches share inside one L2.

template <typename T, int K>
struct WaveFdm {
  T Te[K * K];              // Te[i*K + j]: component i (0..K-1) of symmetric mode j
  T To[(K - 1) * (K - 1)];  // To[i*(K-1) + j]: component i (0..K-2) of antisymmetric mode j
};

// The interior rows of the 2-cell patch mass and stiffness matrices (the
// residual's 1D factors), held as one cell's matrices: a uniform mesh repeats
// the cell matrix, so the (2K-1) x (2K+1) band has (K+1)^2 distinct entries
// per matrix, and unrolled loops address them at compile time.
template <typename T, int K>
struct PatchBand {
  T m[(K + 1) * (K + 1)];  // cell mass matrix, row-major (entry [K][K] unused)
  T k[(K + 1) * (K + 1)];  // cell stiffness matrix
  T mvv, kvv;              // the middle vertex's diagonal: the sum over both cells
};

// entry (j, z) of the band, interior node j in 1..2K-1, closure node z in j's cells
template <typename T, int K>
__device__ inline T band_at(const T (&c)[(K + 1) * (K + 1)], T vv, int j, int z) {
  constexpr int W = K + 1;
  if (j < K) return c[j * W + z];            // first cell
  if (j > K) return c[(j - K) * W + z - K];  // second cell
  if (z < K) return c[K * W + z];            // middle vertex, first cell
  if (z > K) return c[z - K];                // middle vertex, second cell (its row 0)
  return vv;
}
template <typename T, int K>
__device__ inline T band_m(const PatchBand<T, K>& b, int j, int z) { return band_at<T, K>(b.m, b.mvv, j, z); }
template <typename T, int K>
__device__ inline T band_k(const PatchBand<T, K>& b, int j, int z) { return band_at<T, K>(b.k, b.kvv, j, z); }

// The two cell matrices are symmetric: only their upper triangles travel as
// kernel arguments ((K+1)(K+2)/2 instead of (K+1)^2 scalars per matrix), so
// that more of a kernel's constants stay in scalar registers.
template <typename T, int K>
struct SymBand {
  static constexpr int N = (K + 1) * (K + 2) / 2;
  T m[N];  // upper triangle of the cell mass matrix, row by row
  T k[N];  // ... of the cell stiffness matrix
  T mvv, kvv;  // the middle vertex's diagonal: the sum over both cells
};
__host__ __device__ constexpr int sym_idx(int r, int c, int K) {
  return r <= c ? r * (K + 1) - r * (r - 1) / 2 + (c - r) : c * (K + 1) - c * (c - 1) / 2 + (r - c);
}
// entry (j, z) of the band (interior node j, closure node z in j's cells), as band_at
template <typename T, int K>
__device__ inline T sym_at(const T (&c)[(K + 1) * (K + 2) / 2], T vv, int j, int z) {
  if (j < K) return c[sym_idx(j, z, K)];
  if (j > K) return c[sym_idx(j - K, z - K, K)];
  if (z < K) return c[sym_idx(K, z, K)];
  if (z > K) return c[sym_idx(0, z - K, K)];
  return vv;
}
template <typename T, int K>
__device__ inline T sym_m(const SymBand<T, K>& b, int j, int z) { return sym_at<T, K>(b.m, b.mvv, j, z); }
template <typename T, int K>
__device__ inline T sym_k(const SymBand<T, K>& b, int j, int z) { return sym_at<T, K>(b.k, b.kvv, j, z); }
// from the full cell matrices (upper triangles kept)
template <typename T, int K>
inline void make_sym_band(const PatchBand<T, K>& b, SymBand<T, K>* s) {
  constexpr int W = K + 1;
  for (int r = 0; r < W; ++r)
    for (int c = r; c < W; ++c) {
      s->m[sym_idx(r, c, K)] = b.m[r * W + c];
      s->k[sym_idx(r, c, K)] = b.k[r * W + c];
    }
  s->mvv = b.mvv;
  s->kvv = b.kvv;
}

// Fill a PatchBand from the interior rows (Q x P, row-major) of the 2-cell
// patch matrices; false if they are not two copies of one cell matrix.
template <typename T, int K>
inline bool make_band(const double* Mrows, const double* Krows, PatchBand<T, K>* b) {
  constexpr int P = 2 * K + 1, W = K + 1;
  const double* src[2] = {Mrows, Krows};
  T* dst[2] = {b->m, b->k};
  for (int t = 0; t < 2; ++t) {
    const double* R = src[t];
    T* c = dst[t];
    for (int i = 0; i < W * W; ++i) c[i] = T(0);
    for (int a = 1; a <= K; ++a)
      for (int z = 0; z <= K; ++z)
        if (!(a == K && z == K)) c[a * W + z] = (T)R[(a - 1) * P + z];
    for (int z = 1; z <= K; ++z) c[z] = (T)R[(K - 1) * P + K + z];
    (t == 0 ? b->mvv : b->kvv) = (T)R[(K - 1) * P + K];
    for (int j = K + 1; j < 2 * K; ++j)
      for (int z = K; z <= 2 * K; ++z)
        if ((T)R[(j - 1) * P + z] != c[(j - K) * W + z - K]) return false;
  }
  return true;
}

// 1 / d for an eigenvalue sum of the fast diagonalization (d > 0, far from
// overflow and underflow).  FP32: the hardware reciprocal (1 ulp).  FP64: the
// hardware reciprocal refined by one Newton step r + r (1 - d r), which
// squares its relative error; a few instructions instead of the IEEE
// division sequence (the scaling is applied 343 times per Q4 patch).
template <typename T>
__device__ inline T inv_eig(T d) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_amdgcn_rcpf(d);
  } else {
    const T r = __builtin_amdgcn_rcp(d);
    return fma(r, fma(-d, r, T(1)), r);
  }
}

template <typename T, int K>
__device__ inline void fdm_forward(const WaveFdm<T, K>& f, const T (&v)[2 * K - 1], T (&out)[2 * K - 1]) {
  constexpr int Q = 2 * K - 1, M = K - 1;  // M = index of the middle node
  T e[K], o[K - 1];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    e[i] = v[i] + v[Q - 1 - i];
    o[i] = v[i] - v[Q - 1 - i];
  }
  e[M] = v[M];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    T s = T(0);
#pragma unroll
    for (int i = 0; i < K; ++i) s += f.Te[i * K + j] * e[i];
    out[j] = s;
  }
#pragma unroll
  for (int j = 0; j < K - 1; ++j) {
    T s = T(0);
#pragma unroll
    for (int i = 0; i < K - 1; ++i) s += f.To[i * (K - 1) + j] * o[i];
    out[K + j] = s;
  }
}

template <typename T, int K>
__device__ inline void fdm_backward(const WaveFdm<T, K>& f, const T (&c)[2 * K - 1], T (&out)[2 * K - 1]) {
  constexpr int Q = 2 * K - 1, M = K - 1;
  T ce[K], co[K - 1];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    T s = T(0);
#pragma unroll
    for (int j = 0; j < K; ++j) s += f.Te[i * K + j] * c[j];
    ce[i] = s;
  }
#pragma unroll
  for (int i = 0; i < K - 1; ++i) {
    T s = T(0);
#pragma unroll
    for (int j = 0; j < K - 1; ++j) s += f.To[i * (K - 1) + j] * c[K + j];
    co[i] = s;
  }
#pragma unroll
  for (int i = 0; i < M; ++i) {
    out[i] = ce[i] + co[i];
    out[Q - 1 - i] = ce[i] - co[i];
  }
  out[M] = ce[M];
}

template <typename T, int K>
struct WaveArgs {
  T* __restrict__ u;
  const T* __restrict__ b;
  int n1;
  int v0[3];
  int np[3];
  unsigned npatch;
  unsigned vec_bytes;  // bytes of one level vector (< 2^32)
  unsigned magic_x, magic_y;  // magic_of(np[0]), magic_of(np[1]) (see div_magic)
  // order in which the workgroups visit the color's patches (dispatch-order study):
  // 0 lexicographic in one slab per XCD, 1 lexicographic dealt round-robin over the XCDs,
  // 2 Morton curve over a 2^cover_log2 cube in one slab per XCD, 3 tiles of 4^3 patches in one slab per XCD
  int order;
  int cover_log2;
  unsigned nslots;  // workgroups of the launch that map to a position (before the range check)
  int tiles_x, tiles_y;
  PatchBand<T, K> band;  // interior rows of the 2-cell patch mass and stiffness matrices
  WaveFdm<T, K> f;
  T lam[2 * K - 1];  // 1D generalized eigenvalues in the internal mode order
};

template <int K>
__device__ inline void boundary_column(int lane, int& y, int& x) {
  constexpr int P = 2 * K + 1;
  if (lane < P) { y = 0; x = lane; }
  else if (lane < 2 * P) { y = P - 1; x = lane - P; }
  else { const int r = lane - 2 * P; y = 1 + (r >> 1); x = (r & 1) ? P - 1 : 0; }
}

// n / d for a divisor d of the launch: umulhi(n, floor(2^32 / d) + 1) is exact
// for n * d < 2^32 and d >= 2; d = 1 (whose multiplier 2^32 + 1 does not fit)
// is taken apart.
__device__ inline unsigned div_magic(unsigned n, unsigned d, unsigned magic) {
  return d == 1u ? n : __umulhi(n, magic);
}
__host__ inline unsigned magic_of(unsigned d) { return d >= 2u ? (unsigned)((1ull << 32) / d + 1) : 0u; }

// Raw buffer accesses: a wave-uniform descriptor over a whole level vector,
// a wave-uniform byte offset (SGPR) and a 32-bit per-lane byte offset.
// Out-of-range offsets read 0 and drop the store (hardware range check).
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ inline T buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
  }
}
template <typename T>
__device__ inline void buf_store(T v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
  } else {
    typedef unsigned u32x2 __attribute__((vector_size(8)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff, 0);
  }
}

// Global accesses are organised so that consecutive lanes touch consecutive
// x (this matters more than any other choice measured for this kernel):
// closure columns and right-hand side columns are read plane by plane (the
// right-hand side waits in LDS until the residual is formed), and the back
// transform ends along z so that the new interior is written plane by plane
// (the three 1D transforms of T (x) T (x) T commute).  One wave per patch,
// one wave per workgroup.
template <typename T, int K>
__global__ void __launch_bounds__(64) patch_wave3_kernel(const WaveArgs<T, K> a) {
  constexpr int P = 2 * K + 1, Q = 2 * K - 1, P2 = P * P, Q2 = Q * Q, NB = P2 - Q2;
  __shared__ T Z[2 * Q * P2];      // [t][oz][y][x] after the z contraction; later the FDM buffers
  __shared__ T AE[2 * Q * Q * P];  // [t][oz][oy][x] after the y contraction
  __shared__ T B[Q * Q2];          // right-hand side of the interior, [oz][oy][ox]
  T* W0 = Z;
  T* W1 = Z + Q * Q2;
  static_assert(2 * Q * Q2 <= 2 * Q * P2, "FDM buffers must fit in Z");

  const unsigned h = blockIdx.x;
  const unsigned per = gridDim.x / kXcd;
  const unsigned logical = (a.order == 1) ? h : (h % kXcd) * per + h / kXcd;
  if (logical >= a.nslots) return;
  const int lane = threadIdx.x;
  const unsigned npx = (unsigned)a.np[0], npy = (unsigned)a.np[1];
  int px, py, pz;
  if (a.order <= 1) {
    const unsigned qx = div_magic(logical, npx, a.magic_x);
    const unsigned qy = div_magic(qx, npy, a.magic_y);
    px = (int)(logical - qx * npx);
    py = (int)(qx - qy * npy);
    pz = (int)qy;
  } else if (a.order == 2) {
    auto compact = [](unsigned m) {  // every third bit
      m &= 0x09249249u;
      m = (m ^ (m >> 2)) & 0x030c30c3u;
      m = (m ^ (m >> 4)) & 0x0300f00fu;
      m = (m ^ (m >> 8)) & 0xff0000ffu;
      m = (m ^ (m >> 16)) & 0x000003ffu;
      return m;
    };
    px = (int)compact(logical);
    py = (int)compact(logical >> 1);
    pz = (int)compact(logical >> 2);
  } else {
    const unsigned t = logical >> 6, in = logical & 63u;
    const unsigned tx = t % (unsigned)a.tiles_x, tr = t / (unsigned)a.tiles_x;
    px = (int)(4 * tx + (in & 3u));
    py = (int)(4 * (tr % (unsigned)a.tiles_y) + ((in >> 2) & 3u));
    pz = (int)(4 * (tr / (unsigned)a.tiles_y) + (in >> 4));
  }
  if (px >= a.np[0] || py >= a.np[1] || pz >= a.np[2]) return;
  const unsigned n1 = (unsigned)a.n1;
  const size_t n2 = (size_t)n1 * n1;
  const size_t base = (size_t)(K * (a.v0[0] + 2 * px - 1)) + (size_t)n1 * (size_t)(K * (a.v0[1] + 2 * py - 1)) +
                      n2 * (size_t)(K * (a.v0[2] + 2 * pz - 1));
  const __amdgpu_buffer_rsrc_t ur = make_rsrc(a.u, a.vec_bytes);
  const __amdgpu_buffer_rsrc_t br = make_rsrc(a.b, a.vec_bytes);
  const unsigned sbase = (unsigned)(base * sizeof(T));  // patch origin, bytes
  const unsigned splane = (unsigned)(n2 * sizeof(T));   // one z plane, bytes

  // ---- 0. every global load of the patch, issued before any arithmetic ----
  int by = 0, bx = 0;
  boundary_column<K>(lane < NB ? lane : 0, by, bx);
  T vb[P];
  if (lane < NB) {
    const unsigned off = (n1 * (unsigned)by + (unsigned)bx) * (unsigned)sizeof(T);
#pragma unroll
    for (int z = 0; z < P; ++z) vb[z] = buf_load<T>(ur, off, sbase + splane * z);
  }
  const int iy = 1 + lane / Q, ix = 1 + lane % Q;
  T v0 = T(0), v1 = T(0), bv[Q];
  if (lane < Q2) {
    const unsigned off = (n1 * (unsigned)iy + (unsigned)ix) * (unsigned)sizeof(T);
    v0 = buf_load<T>(ur, off, sbase);
    v1 = buf_load<T>(ur, off, sbase + splane * (P - 1));
#pragma unroll
    for (int o = 0; o < Q; ++o) bv[o] = buf_load<T>(br, off, sbase + splane * (o + 1));
  }
  // ---- 1. z contraction; right-hand side columns into LDS ----
  if (lane < NB) {
#pragma unroll
    for (int o = 0; o < Q; ++o) {
      const int j = o + 1;
      T zm = T(0), zk = T(0);
#pragma unroll
      for (int z = 0; z < P; ++z) {
        if (z < band_lo(j, K) || z > band_hi(j, K)) continue;
        zm = fma(band_m(a.band, j, z), vb[z], zm);
        zk = fma(band_k(a.band, j, z), vb[z], zk);
      }
      Z[(0 * Q + o) * P2 + by * P + bx] = zm;
      Z[(1 * Q + o) * P2 + by * P + bx] = zk;
    }
  }
  if (lane < Q2) {
#pragma unroll
    for (int o = 0; o < Q; ++o) B[o * Q2 + lane] = bv[o];
#pragma unroll
    for (int o = 0; o < Q; ++o) {
      const int j = o + 1;
      T zm = T(0), zk = T(0);
      if (band_lo(j, K) == 0) { zm = fma(band_m(a.band, j, 0), v0, zm); zk = fma(band_k(a.band, j, 0), v0, zk); }
      if (band_hi(j, K) == P - 1) { zm = fma(band_m(a.band, j, P - 1), v1, zm); zk = fma(band_k(a.band, j, P - 1), v1, zk); }
      Z[(0 * Q + o) * P2 + iy * P + ix] = zm;
      Z[(1 * Q + o) * P2 + iy * P + ix] = zk;
    }
  }
  __syncthreads();

  // ---- 2. y contraction: A = M_y Zm, E = K_y Zm + M_y Zk ----
  if (lane < Q * P) {
    const int oz = lane / P, x = lane % P;
    T zm[P], zk[P];
#pragma unroll
    for (int y = 0; y < P; ++y) {
      zm[y] = Z[(0 * Q + oz) * P2 + y * P + x];
      zk[y] = Z[(1 * Q + oz) * P2 + y * P + x];
    }
#pragma unroll
    for (int o = 0; o < Q; ++o) {
      const int j = o + 1;
      T av = T(0), ev = T(0);
#pragma unroll
      for (int y = 0; y < P; ++y) {
        if (y < band_lo(j, K) || y > band_hi(j, K)) continue;
        av = fma(band_m(a.band, j, y), zm[y], av);
        ev = fma(band_k(a.band, j, y), zm[y], ev);
        ev = fma(band_m(a.band, j, y), zk[y], ev);
      }
      AE[((0 * Q + oz) * Q + o) * P + x] = av;
      AE[((1 * Q + oz) * Q + o) * P + x] = ev;
    }
  }
  __syncthreads();

  // ---- 3. x contraction, local residual, T^T along x  (lanes (oz, oy)) ----
  if (lane < Q2) {
    const int oz = lane / Q, oy = lane % Q;
    T av[P], ev[P];
#pragma unroll
    for (int x = 0; x < P; ++x) {
      av[x] = AE[((0 * Q + oz) * Q + oy) * P + x];
      ev[x] = AE[((1 * Q + oz) * Q + oy) * P + x];
    }
    T r[Q], m[Q];
#pragma unroll
    for (int o = 0; o < Q; ++o) {
      const int j = o + 1;
      T s = T(0);
#pragma unroll
      for (int x = 0; x < P; ++x) {
        if (x < band_lo(j, K) || x > band_hi(j, K)) continue;
        s = fma(band_k(a.band, j, x), av[x], s);
        s = fma(band_m(a.band, j, x), ev[x], s);
      }
      r[o] = B[oz * Q2 + oy * Q + o] - s;
    }
    fdm_forward<T, K>(a.f, r, m);
#pragma unroll
    for (int j = 0; j < Q; ++j) W0[(oz * Q + oy) * Q + j] = m[j];
  }
  __syncthreads();

  // ---- 4. T^T along y  (lanes (oz, mx)) ----
  if (lane < Q2) {
    const int oz = lane / Q, mx = lane % Q;
    T v[Q], m[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = W0[(oz * Q + i) * Q + mx];
    fdm_forward<T, K>(a.f, v, m);
#pragma unroll
    for (int j = 0; j < Q; ++j) W1[(oz * Q + j) * Q + mx] = m[j];
  }
  __syncthreads();

  // ---- 5. T^T along z and 1/Lambda  (lanes (my, mx)) ----
  if (lane < Q2) {
    const int my = lane / Q, mx = lane % Q;
    T v[Q], c[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = W1[(i * Q + my) * Q + mx];
    fdm_forward<T, K>(a.f, v, c);
#pragma unroll
    for (int j = 0; j < Q; ++j)
      {
        T lmy = a.lam[0], lmx = a.lam[0];
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          lmy = (my == i) ? a.lam[i] : lmy;
          lmx = (mx == i) ? a.lam[i] : lmx;
        }
        const T s2 = lmy + lmx;
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          W0[(j * Q + my) * Q + mx] = c[j] * inv_eig(s2 + a.lam[j]);
        }
      }
  }
  __syncthreads();
  // ---- 6. T along x  (lanes (mz, my)) ----
  if (lane < Q2) {
    const int mz = lane / Q, my = lane % Q;
    T c[Q], d[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) c[j] = W0[(mz * Q + my) * Q + j];
    fdm_backward<T, K>(a.f, c, d);
#pragma unroll
    for (int i = 0; i < Q; ++i) W1[(mz * Q + my) * Q + i] = d[i];
  }
  __syncthreads();
  // ---- 7. T along y  (lanes (mz, x)) ----
  if (lane < Q2) {
    const int mz = lane / Q, x = lane % Q;
    T c[Q], d[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) c[j] = W1[(mz * Q + j) * Q + x];
    fdm_backward<T, K>(a.f, c, d);
#pragma unroll
    for (int i = 0; i < Q; ++i) W0[(mz * Q + i) * Q + x] = d[i];
  }
  __syncthreads();
  // ---- 8. T along z, store the new interior plane by plane  (lanes (y, x)) ----
  if (lane < Q2) {
    T c[Q], d[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) c[j] = W0[j * Q2 + lane];
    fdm_backward<T, K>(a.f, c, d);
    const int y = 1 + lane / Q, x = 1 + lane % Q;
    const unsigned off = (n1 * (unsigned)y + (unsigned)x) * (unsigned)sizeof(T);
#pragma unroll
    for (int i = 0; i < Q; ++i) buf_store<T>(d[i], ur, off, sbase + splane * (i + 1));
  }
}

}  // namespace vps
