// Patch smoother kernel for 2D, constant coefficient: a row of x-adjacent
// patches of one color per wavefront.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "patch_wave.h"

namespace vps {

// ---------------------------------------------------------------------------
// Same update as the 3D one-patch kernel (exact local solve from the closure
// with the interior values taken as zero, fast diagonalisation in even/odd
// form), in 2D.  Same-color patches 2 vertices apart along x have closures
// that share a face column, so G of them side by side span G*2K + 1 node
// columns: one lane per column loads the closure rows as contiguous runs of
// up to 61 values, and the y direction stays in the lane's registers.
//
// Stages of the wave that owns G patches of one color row:
//   1. lanes = closure columns: every load (closure rows of u; the
//      right-hand side into the lanes (patch, interior column)), y
//      contraction of the column (interior rows taken as zero off the face
//      columns); the right-hand side into LDS;
//   2. lanes = (patch, interior row): x contraction of the row from LDS,
//      local residual, T^T along x in registers;
//   3. lanes = (patch, x mode): T^T along y, 1/Lambda;
//   4. lanes = (patch, y mode): T along x;
//   5. lanes = (patch, interior column): T along y, store the column.
// Each lane keeps one line in registers at a time; between stages the lines
// change direction through LDS.

template <int K>
struct RowShape {
  static constexpr int P = 2 * K + 1, Q = 2 * K - 1, S = 2 * K;
  static constexpr int G = 63 / S;   // patches per wave
  static constexpr int C = G * S + 1;  // closure columns of the G patches
  static_assert(C <= 64 && G * Q <= 64, "a row of patches must fit one wave");
};

template <typename T, int K>
struct RowArgs {
  T* __restrict__ u;
  const T* __restrict__ b;
  int n1;
  int v0[2];
  int np[2];
  int ngx;             // groups of G patches per color row: ceil(np[0] / G)
  unsigned ngroups;    // ngx * np[1]
  unsigned vec_bytes;  // bytes of one level vector (< 2^32)
  unsigned magic_g;    // magic_of(ngx) (see div_magic)
  PatchBand<T, K> band;  // interior rows of the 2-cell patch mass and stiffness matrices
  WaveFdm<T, K> f;
  T lam[2 * K - 1];  // 1D generalized eigenvalues in the internal mode order
};

template <typename T, int K>
__global__ void __launch_bounds__(64) patch_row2_kernel(const RowArgs<T, K> a) {
  using R = RowShape<K>;
  constexpr int P = R::P, Q = R::Q, S = R::S, G = R::G, C = R::C, GQ = G * Q, Q2 = Q * Q;
  __shared__ T ZM[Q * C];    // [oy][column] after the y contraction: M_y u
  __shared__ T ZK[Q * C];    // ... and K_y u
  __shared__ T W[G * Q2];    // [patch][.][.]: right-hand side, then the transposes of the FDM

  const unsigned h = blockIdx.x;
  const unsigned per = gridDim.x / kXcd;
  const unsigned g = (h % kXcd) * per + h / kXcd;  // one contiguous slab of groups per XCD
  if (g >= a.ngroups) return;
  const int lane = threadIdx.x;
  const unsigned ngx = (unsigned)a.ngx;
  const unsigned qy = div_magic(g, ngx, a.magic_g);
  const int px0 = G * (int)(g - qy * ngx);
  const int py = (int)qy;
  const int nact = min(G, a.np[0] - px0);  // patches of the group that exist
  const int cmax = nact * S;               // last closure column that exists
  const unsigned n1 = (unsigned)a.n1;
  const size_t base = (size_t)(K * (a.v0[0] + 2 * px0 - 1)) + (size_t)n1 * (size_t)(K * (a.v0[1] + 2 * py - 1));
  const __amdgpu_buffer_rsrc_t ur = make_rsrc(a.u, a.vec_bytes);
  const __amdgpu_buffer_rsrc_t br = make_rsrc(a.b, a.vec_bytes);
  const unsigned sbase = (unsigned)(base * sizeof(T));
  const unsigned srow = n1 * (unsigned)sizeof(T);

  // ---- every global load, before any arithmetic (lanes past a list repeat an
  //      entry that exists, so every load is unconditional) ----
  const int col = min(lane, cmax);
  T uc[P];
#pragma unroll
  for (int y = 0; y < P; ++y) uc[y] = buf_load<T>(ur, (unsigned)col * (unsigned)sizeof(T), sbase + srow * y);
  const int l2 = min(lane, GQ - 1);
  const int pp = l2 / Q, ll = l2 % Q;  // (patch, line) of stages 2-5
  const unsigned off2 = (unsigned)min(pp * S + 1 + ll, cmax) * (unsigned)sizeof(T);
  T bv[Q];
#pragma unroll
  for (int o = 0; o < Q; ++o) bv[o] = buf_load<T>(br, off2, sbase + srow * (o + 1));

  // ---- 1. y contraction of the closure columns; right-hand side into W[p][oy][ox] ----
  if (lane < C) {
    if (lane % S != 0) {  // a column inside a patch: its interior rows count as zero
#pragma unroll
      for (int y = 1; y < P - 1; ++y) uc[y] = T(0);
    }
#pragma unroll
    for (int o = 0; o < Q; ++o) {
      const int j = o + 1;
      T zm = T(0), zk = T(0);
#pragma unroll
      for (int y = 0; y < P; ++y) {
        if (y < band_lo(j, K) || y > band_hi(j, K)) continue;
        zm = fma(band_m(a.band, j, y), uc[y], zm);
        zk = fma(band_k(a.band, j, y), uc[y], zk);
      }
      ZM[o * C + lane] = zm;
      ZK[o * C + lane] = zk;
    }
  }
  if (lane < GQ) {
#pragma unroll
    for (int o = 0; o < Q; ++o) W[(pp * Q + o) * Q + ll] = bv[o];
  }
  __syncthreads();

  // ---- 2. x contraction of row oy, local residual, T^T along x  (lanes (patch, oy)) ----
  if (lane < GQ) {
    const int oy = ll, c0 = pp * S;
    T zm[P], zk[P], r[Q], m[Q];
#pragma unroll
    for (int x = 0; x < P; ++x) {
      zm[x] = ZM[oy * C + c0 + x];
      zk[x] = ZK[oy * C + c0 + x];
    }
#pragma unroll
    for (int o = 0; o < Q; ++o) {
      const int j = o + 1;
      T acc = T(0);
#pragma unroll
      for (int x = 0; x < P; ++x) {
        if (x < band_lo(j, K) || x > band_hi(j, K)) continue;
        acc = fma(band_k(a.band, j, x), zm[x], acc);
        acc = fma(band_m(a.band, j, x), zk[x], acc);
      }
      r[o] = W[(pp * Q + oy) * Q + o] - acc;
    }
    fdm_forward<T, K>(a.f, r, m);
#pragma unroll
    for (int q = 0; q < Q; ++q) W[(pp * Q + oy) * Q + q] = m[q];  // the lane's own row: [p][oy][mx]
  }
  __syncthreads();

  // ---- 3. T^T along y, 1/Lambda  (lanes (patch, mx)) ----
  if (lane < GQ) {
    const int mx = ll;
    T v[Q], c[Q];
#pragma unroll
    for (int y = 0; y < Q; ++y) v[y] = W[(pp * Q + y) * Q + mx];
    fdm_forward<T, K>(a.f, v, c);
    T lmx = a.lam[0];
#pragma unroll
    for (int q = 1; q < Q; ++q) lmx = (mx == q) ? a.lam[q] : lmx;
#pragma unroll
    for (int q = 0; q < Q; ++q) {  // the lane's own column: [p][my][mx]
      W[(pp * Q + q) * Q + mx] = c[q] * inv_eig(lmx + a.lam[q]);
    }
  }
  __syncthreads();

  // ---- 4. T along x  (lanes (patch, my)) ----
  if (lane < GQ) {
    const int my = ll;
    T c[Q], d[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) c[q] = W[(pp * Q + my) * Q + q];
    fdm_backward<T, K>(a.f, c, d);
#pragma unroll
    for (int x = 0; x < Q; ++x) W[(pp * Q + my) * Q + x] = d[x];  // the lane's own row: [p][my][x]
  }
  __syncthreads();

  // ---- 5. T along y, store the new interior column  (lanes (patch, x)) ----
  if (lane < GQ) {
    const int x = ll;
    T c[Q], d[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) c[q] = W[(pp * Q + q) * Q + x];
    fdm_backward<T, K>(a.f, c, d);
    if (pp < nact) {
#pragma unroll
      for (int y = 0; y < Q; ++y) buf_store<T>(d[y], ur, off2, sbase + srow * (y + 1));
    }
  }
}

}  // namespace vps
