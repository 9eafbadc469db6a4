// Patch smoother kernel for 3D, constant coefficient, one patch per wavefront
// for degrees whose (2K-1)^2 interior lines exceed the 64 lanes (K = 5).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "patch_wave.h"

namespace vps {

// ---------------------------------------------------------------------------
// The update of patch_wave3_kernel (exact local solve from the closure with
// the interior values taken as zero, fast diagonalisation in even/odd form)
// with every stage that has more lines than lanes run in passes of 64.  The
// residual contracts z, x, y (the last in lanes (z, x) over y), so the
// right-hand side is loaded straight into the lanes that subtract it and
// needs no LDS; the x contraction writes its outputs over its own inputs
// (each lane owns one (z, y) line of both arrays), which keeps the LDS at
// 2 (2K-1)(2K+1)^2 values (17.4 KB in FP64 at K = 5: 9 waves per CU fit, the
// registers allow 8).
//
// Stages:  0. every global load (boundary columns along z, the two end values
// of the interior columns, the right-hand side rows);  1. z contraction;
// 2. x contraction of the (z-out, y) lines;  3. y contraction, local residual,
// T^T along y;  4. T^T along x;  5. T^T along z and 1/Lambda;  6. T along x;
// 7. T along y;  8. T along z and store, plane by plane.

template <typename T, int K>
struct BigArgs {
  T* __restrict__ u;
  const T* __restrict__ b;
  int n1;
  int v0[3];
  int np[3];
  unsigned npatch;
  unsigned vec_bytes;         // bytes of one level vector (< 2^32)
  unsigned magic_x, magic_y;  // magic_of(np[0]), magic_of(np[1]) (see div_magic)
  SymBand<T, K> band;         // interior rows of the 2-cell patch mass and stiffness matrices
  WaveFdm<T, K> f;
  T lam[2 * K - 1];  // 1D generalized eigenvalues in the internal mode order
};
// The FDM factors and eigenvalues (50 scalars at K = 5) are read from LDS: with
// the band coefficients they would not fit the scalar registers, and FP64
// constants spilled to vector lanes cost two lane reads per use.
template <typename T, int K>
struct BigFdm {
  WaveFdm<T, K> f;
  T lam[2 * K - 1];
};

template <typename T, int K>
__global__ void __launch_bounds__(64) patch_big3_kernel(const BigArgs<T, K> a) {
  constexpr int P = 2 * K + 1, Q = 2 * K - 1, P2 = P * P, Q2 = Q * Q, Q3 = Q * Q2, NB = P2 - Q2;
  constexpr int NL = (Q2 + 63) / 64;     // passes over the Q^2 lines
  constexpr int NX = (Q * P + 63) / 64;  // passes over the Q P lines of the x contraction
  static_assert(NB <= 64, "the boundary columns must fit one wave");
  __shared__ T Z[2 * Q * P2];  // [t][oz][y][x] after the z contraction, [t][oz][y][ox] (ox < Q) after the
                               // x contraction (in place); later the FDM buffers
  __shared__ BigFdm<T, K> FS;
  T* W0 = Z;
  T* W1 = Z + Q3;
  static_assert(2 * Q3 <= 2 * Q * P2, "FDM buffers must fit in Z");

  const unsigned h = blockIdx.x;
  const unsigned per = gridDim.x / kXcd;
  const unsigned logical = (h % kXcd) * per + h / kXcd;  // one contiguous slab of patches per XCD
  if (logical >= a.npatch) return;
  const int lane = threadIdx.x;
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < K * K; ++q) FS.f.Te[q] = a.f.Te[q];
#pragma unroll
    for (int q = 0; q < (K - 1) * (K - 1); ++q) FS.f.To[q] = a.f.To[q];
#pragma unroll
    for (int q = 0; q < Q; ++q) FS.lam[q] = a.lam[q];
  }
  const unsigned npx = (unsigned)a.np[0], npy = (unsigned)a.np[1];
  const unsigned qx = div_magic(logical, npx, a.magic_x);
  const unsigned qy = div_magic(qx, npy, a.magic_y);
  const int px = (int)(logical - qx * npx);
  const int py = (int)(qx - qy * npy);
  const int pz = (int)qy;
  const unsigned n1 = (unsigned)a.n1;
  const size_t n2 = (size_t)n1 * n1;
  const size_t base = (size_t)(K * (a.v0[0] + 2 * px - 1)) + (size_t)n1 * (size_t)(K * (a.v0[1] + 2 * py - 1)) +
                      n2 * (size_t)(K * (a.v0[2] + 2 * pz - 1));
  const __amdgpu_buffer_rsrc_t ur = make_rsrc(a.u, a.vec_bytes);
  const __amdgpu_buffer_rsrc_t br = make_rsrc(a.b, a.vec_bytes);
  const unsigned sbase = (unsigned)(base * sizeof(T));
  const unsigned splane = (unsigned)(n2 * sizeof(T));
  const unsigned srow = n1 * (unsigned)sizeof(T);

  // ---- 0. every global load, issued before any arithmetic (lanes past a list
  //      repeat its last entry, so every load is unconditional) ----
  int by, bx;
  boundary_column<K>(min(lane, NB - 1), by, bx);
  T vb[P];
  {
    const unsigned off = srow * (unsigned)by + (unsigned)bx * (unsigned)sizeof(T);
#pragma unroll
    for (int z = 0; z < P; ++z) vb[z] = buf_load<T>(ur, off, sbase + splane * z);
  }
  // interior columns (y, x) and right-hand side lines (z, x) over y: item i -> (i / Q, i % Q)
  T e0[NL], e1[NL], bv[NL][Q];
#pragma unroll
  for (int s = 0; s < NL; ++s) {
    const int i = min(lane + 64 * s, Q2 - 1);
    const int r = i / Q, c = i % Q;
    const unsigned offc = srow * (unsigned)(1 + r) + (unsigned)(1 + c) * (unsigned)sizeof(T);
    e0[s] = buf_load<T>(ur, offc, sbase);
    e1[s] = buf_load<T>(ur, offc, sbase + splane * (P - 1));
    const unsigned offb = splane * (unsigned)(1 + r) + srow + (unsigned)(1 + c) * (unsigned)sizeof(T);
#pragma unroll
    for (int o = 0; o < Q; ++o) bv[s][o] = buf_load<T>(br, offb, sbase + srow * (unsigned)o);
  }

  // ---- 1. z contraction ----
  if (lane < NB) {
#pragma unroll
    for (int o = 0; o < Q; ++o) {
      const int j = o + 1;
      T zm = T(0), zk = T(0);
#pragma unroll
      for (int z = 0; z < P; ++z) {
        if (z < band_lo(j, K) || z > band_hi(j, K)) continue;
        zm = fma(sym_m(a.band, j, z), vb[z], zm);
        zk = fma(sym_k(a.band, j, z), vb[z], zk);
      }
      Z[(0 * Q + o) * P2 + by * P + bx] = zm;
      Z[(1 * Q + o) * P2 + by * P + bx] = zk;
    }
  }
#pragma unroll
  for (int s = 0; s < NL; ++s) {
    const int i = lane + 64 * s;
    if (i < Q2) {
      const int col = (1 + i / Q) * P + 1 + i % Q;
#pragma unroll
      for (int o = 0; o < Q; ++o) {
        const int j = o + 1;
        T zm = T(0), zk = T(0);
        if (band_lo(j, K) == 0) { zm = fma(sym_m(a.band, j, 0), e0[s], zm); zk = fma(sym_k(a.band, j, 0), e0[s], zk); }
        if (band_hi(j, K) == P - 1) { zm = fma(sym_m(a.band, j, P - 1), e1[s], zm); zk = fma(sym_k(a.band, j, P - 1), e1[s], zk); }
        Z[(0 * Q + o) * P2 + col] = zm;
        Z[(1 * Q + o) * P2 + col] = zk;
      }
    }
  }
  __syncthreads();

  // ---- 2. x contraction: A = M_x Zm, E = K_x Zm + M_x Zk  (lines (oz, y)) ----
#pragma unroll
  for (int s = 0; s < NX; ++s) {
    const int i = lane + 64 * s;
    if (i < Q * P) {
      const int oz = i / P, y = i % P;
      T zm[P], zk[P];
#pragma unroll
      for (int x = 0; x < P; ++x) {
        zm[x] = Z[(0 * Q + oz) * P2 + y * P + x];
        zk[x] = Z[(1 * Q + oz) * P2 + y * P + x];
      }
#pragma unroll
      for (int o = 0; o < Q; ++o) {
        const int j = o + 1;
        T av = T(0), ev = T(0);
#pragma unroll
        for (int x = 0; x < P; ++x) {
          if (x < band_lo(j, K) || x > band_hi(j, K)) continue;
          av = fma(sym_m(a.band, j, x), zm[x], av);
          ev = fma(sym_k(a.band, j, x), zm[x], ev);
          ev = fma(sym_m(a.band, j, x), zk[x], ev);
        }
        Z[(0 * Q + oz) * P2 + y * P + o] = av;  // over this lane's own line (read above)
        Z[(1 * Q + oz) * P2 + y * P + o] = ev;
      }
    }
  }
  __syncthreads();

  // ---- 3. y contraction, local residual, T^T along y  (lines (oz, ox)); the
  //      results wait in registers until every lane has read its inputs, which
  //      lie where W0 goes ----
  T mres[NL][Q];
#pragma unroll
  for (int s = 0; s < NL; ++s) {
    const int i = lane + 64 * s;
    if (i < Q2) {
      const int oz = i / Q, ox = i % Q;
      T av[P], ev[P];
#pragma unroll
      for (int y = 0; y < P; ++y) {
        av[y] = Z[(0 * Q + oz) * P2 + y * P + ox];
        ev[y] = Z[(1 * Q + oz) * P2 + y * P + ox];
      }
      T r[Q];
#pragma unroll
      for (int o = 0; o < Q; ++o) {
        const int j = o + 1;
        T acc = T(0);
#pragma unroll
        for (int y = 0; y < P; ++y) {
          if (y < band_lo(j, K) || y > band_hi(j, K)) continue;
          acc = fma(sym_k(a.band, j, y), av[y], acc);
          acc = fma(sym_m(a.band, j, y), ev[y], acc);
        }
        r[o] = bv[s][o] - acc;
      }
      fdm_forward<T, K>(FS.f, r, mres[s]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NL; ++s) {
    const int i = lane + 64 * s;
    if (i < Q2) {
      const int oz = i / Q, ox = i % Q;
#pragma unroll
      for (int q = 0; q < Q; ++q) W0[(oz * Q + q) * Q + ox] = mres[s][q];
    }
  }
  __syncthreads();

  // ---- 4. T^T along x  (lines (oz, my)) ----
#pragma unroll
  for (int s = 0; s < NL; ++s) {
    const int i = lane + 64 * s;
    if (i < Q2) {
      T v[Q], m[Q];
#pragma unroll
      for (int x = 0; x < Q; ++x) v[x] = W0[i * Q + x];
      fdm_forward<T, K>(FS.f, v, m);
#pragma unroll
      for (int q = 0; q < Q; ++q) W1[i * Q + q] = m[q];
    }
  }
  __syncthreads();

  // ---- 5. T^T along z and 1/Lambda  (lines (my, mx)) ----
#pragma unroll
  for (int s = 0; s < NL; ++s) {
    const int i = lane + 64 * s;
    if (i < Q2) {
      const int my = i / Q, mx = i % Q;
      T v[Q], c[Q];
#pragma unroll
      for (int z = 0; z < Q; ++z) v[z] = W1[z * Q2 + i];
      fdm_forward<T, K>(FS.f, v, c);
      T lmy = FS.lam[0], lmx = FS.lam[0];
#pragma unroll
      for (int q = 1; q < Q; ++q) {
        lmy = (my == q) ? FS.lam[q] : lmy;
        lmx = (mx == q) ? FS.lam[q] : lmx;
      }
      const T s2 = lmy + lmx;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        W0[q * Q2 + i] = c[q] * inv_eig(s2 + FS.lam[q]);
      }
    }
  }
  __syncthreads();

  // ---- 6. T along x  (lines (mz, my)) ----
#pragma unroll
  for (int s = 0; s < NL; ++s) {
    const int i = lane + 64 * s;
    if (i < Q2) {
      T c[Q], d[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) c[q] = W0[i * Q + q];
      fdm_backward<T, K>(FS.f, c, d);
#pragma unroll
      for (int x = 0; x < Q; ++x) W1[i * Q + x] = d[x];
    }
  }
  __syncthreads();

  // ---- 7. T along y  (lines (mz, x)) ----
#pragma unroll
  for (int s = 0; s < NL; ++s) {
    const int i = lane + 64 * s;
    if (i < Q2) {
      const int mz = i / Q, x = i % Q;
      T c[Q], d[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) c[q] = W1[(mz * Q + q) * Q + x];
      fdm_backward<T, K>(FS.f, c, d);
#pragma unroll
      for (int y = 0; y < Q; ++y) W0[(mz * Q + y) * Q + x] = d[y];
    }
  }
  __syncthreads();

  // ---- 8. T along z, store the new interior plane by plane  (lines (y, x)) ----
#pragma unroll
  for (int s = 0; s < NL; ++s) {
    const int i = lane + 64 * s;
    if (i < Q2) {
      T c[Q], d[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) c[q] = W0[q * Q2 + i];
      fdm_backward<T, K>(FS.f, c, d);
      const unsigned off = srow * (unsigned)(1 + i / Q) + (unsigned)(1 + i % Q) * (unsigned)sizeof(T);
#pragma unroll
      for (int z = 0; z < Q; ++z) buf_store<T>(d[z], ur, off, sbase + splane * (z + 1));
    }
  }
}

}  // namespace vps
