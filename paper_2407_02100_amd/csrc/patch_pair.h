// Patch smoother kernel for 3D, constant coefficient: two x-adjacent patches
// of one color per wavefront.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "patch_wave.h"

namespace vps {

// ---------------------------------------------------------------------------
// Same update as patch_wave3_kernel (exact local solve from the closure with
// the interior values taken as zero, fast diagonalisation in even/odd form),
// for the patches px0 = 2g and px0 + 1 of a color row along x.  Their
// closures share the node plane x = 2K (pair coordinates), so the boundary
// columns of both closures, (4K+1) x (2K+1) minus the interiors, are loaded
// by one set of wave-wide loads along z: rows of 4K+1 values instead of two
// rows of 2K+1, about a third fewer cache lines and load instructions for the
// boundary, which is most of what the one-patch kernel is bound by (the
// per-CU vector-memory path).  Every load of both patches is issued first;
// the two patches are then solved one after the other with the one-patch
// LDS footprint, the second patch's loads landing while the first computes.
//
// The contractions of the local residual go z, x, y (the last one in lanes
// (z, x) over y), so that the right-hand side is loaded straight into the
// lanes that subtract it (x-z rows of the interior, as coalesced as x-y rows)
// and needs no LDS.
//
// Stages per patch:
//   1. z contraction of its closure columns;  2. x contraction of the
//   (z-out, y) lines;  3. y contraction, local residual, T^T along y;
//   4. T^T along x;  5. T^T along z and 1/Lambda;  6. T along x;
//   7. T along y;  8. T along z and store, plane by plane.
// The last pair of an odd row has one patch: the other's loads are clamped
// into the first closure and it is not solved.

template <typename T, int K>
struct PairArgs {
  T* __restrict__ u;
  const T* __restrict__ b;
  int n1;
  int v0[3];
  int np[3];
  int ngx;             // pairs per color row along x: ceil(np[0] / 2)
  unsigned ngroups;    // ngx * np[1] * np[2]
  unsigned vec_bytes;  // bytes of one level vector (< 2^32)
  unsigned magic_g, magic_y;  // magic_of(ngx), magic_of(np[1]) (see div_magic)
  PatchBand<T, K> band;  // interior rows of the 2-cell patch mass and stiffness matrices
  WaveFdm<T, K> f;
  T lam[2 * K - 1];  // 1D generalized eigenvalues in the internal mode order
};

template <typename T, int K>
__global__ void __launch_bounds__(64) patch_pair3_kernel(const PairArgs<T, K> a) {
  constexpr int P = 2 * K + 1, Q = 2 * K - 1, P2 = P * P, Q2 = Q * Q;
  constexpr int UW = 2 * P - 1;        // width of the pair's closures along x
  constexpr int NBU = 2 * UW + 3 * Q;  // boundary columns of the two closures
  static_assert(NBU <= 64 && Q * P <= 64, "one wave per pair needs the boundary columns in 64 lanes");
  __shared__ T Z[2 * Q * P2];      // [t][oz][y][x] after the z contraction; later the FDM buffers
  __shared__ T AE[2 * Q * P * Q];  // [t][oz][y][ox] after the x contraction
  T* W0 = Z;
  T* W1 = Z + Q * Q2;
  static_assert(2 * Q * Q2 <= 2 * Q * P2, "FDM buffers must fit in Z");

  const unsigned h = blockIdx.x;
  const unsigned per = gridDim.x / kXcd;
  const unsigned g = (h % kXcd) * per + h / kXcd;  // one contiguous slab of pairs per XCD
  if (g >= a.ngroups) return;
  const int lane = threadIdx.x;
  const unsigned ngx = (unsigned)a.ngx, npy = (unsigned)a.np[1];
  const unsigned qx = div_magic(g, ngx, a.magic_g);
  const unsigned qy = div_magic(qx, npy, a.magic_y);
  const int px0 = 2 * (int)(g - qx * ngx);
  const int py = (int)(qx - qy * npy);
  const int pz = (int)qy;
  const int nact = min(2, a.np[0] - px0);  // patches of the pair that exist
  const int xmax = nact * (P - 1);         // last pair column that exists
  const unsigned n1 = (unsigned)a.n1;
  const size_t n2 = (size_t)n1 * n1;
  const size_t base = (size_t)(K * (a.v0[0] + 2 * px0 - 1)) + (size_t)n1 * (size_t)(K * (a.v0[1] + 2 * py - 1)) +
                      n2 * (size_t)(K * (a.v0[2] + 2 * pz - 1));
  const __amdgpu_buffer_rsrc_t ur = make_rsrc(a.u, a.vec_bytes);
  const __amdgpu_buffer_rsrc_t br = make_rsrc(a.b, a.vec_bytes);
  const unsigned sbase = (unsigned)(base * sizeof(T));  // pair origin, bytes
  const unsigned splane = (unsigned)(n2 * sizeof(T));   // one z plane, bytes
  const unsigned srow = n1 * (unsigned)sizeof(T);       // one y row, bytes

  // ---- every global load of the pair, issued before any arithmetic (lanes
  //      past a list repeat its last entry, so every load is unconditional) ----
  // boundary columns (y, x) of the two closures, x in [0, 4K]
  int by, bx;
  {
    const int l = min(lane, NBU - 1);
    if (l < UW) { by = 0; bx = l; }
    else if (l < 2 * UW) { by = P - 1; bx = l - UW; }
    else { const int r = l - 2 * UW; by = 1 + r / 3; bx = (r % 3) * (P - 1); }
  }
  T vb[P];
  {
    const unsigned off = srow * (unsigned)by + (unsigned)min(bx, xmax) * (unsigned)sizeof(T);
#pragma unroll
    for (int z = 0; z < P; ++z) vb[z] = buf_load<T>(ur, off, sbase + splane * z);
  }
  // per patch: the end values of its interior columns (lanes (y, x)) and its
  // right-hand side in lanes (z, x), over y
  const int la = min(lane, Q2 - 1);
  const int ly = la / Q, lx = la % Q;
  T e0[2], e1[2], bv[2][Q];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const int x = min(1 + lx + p * (P - 1), xmax);
    const unsigned offc = srow * (unsigned)(1 + ly) + (unsigned)x * (unsigned)sizeof(T);
    e0[p] = buf_load<T>(ur, offc, sbase);
    e1[p] = buf_load<T>(ur, offc, sbase + splane * (P - 1));
    const unsigned offb = splane * (unsigned)(1 + ly) + srow + (unsigned)x * (unsigned)sizeof(T);  // lane offsets
#pragma unroll
    for (int o = 0; o < Q; ++o) bv[p][o] = buf_load<T>(br, offb, sbase + srow * (unsigned)o);
  }

#pragma unroll
  for (int p = 0; p < 2; ++p) {
    if (p == 1) {
      if (nact < 2) break;
      __syncthreads();  // the first patch's last LDS reads are done
    }
    const int x0 = p * (P - 1);  // the patch's first column in pair coordinates

    // ---- 1. z contraction of the patch's closure columns ----
    if (lane < NBU && bx >= x0 && bx <= x0 + P - 1) {
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
        Z[(0 * Q + o) * P2 + by * P + bx - x0] = zm;
        Z[(1 * Q + o) * P2 + by * P + bx - x0] = zk;
      }
    }
    if (lane < Q2) {
      const int col = (1 + ly) * P + 1 + lx;
#pragma unroll
      for (int o = 0; o < Q; ++o) {
        const int j = o + 1;
        T zm = T(0), zk = T(0);
        if (band_lo(j, K) == 0) { zm = fma(band_m(a.band, j, 0), e0[p], zm); zk = fma(band_k(a.band, j, 0), e0[p], zk); }
        if (band_hi(j, K) == P - 1) { zm = fma(band_m(a.band, j, P - 1), e1[p], zm); zk = fma(band_k(a.band, j, P - 1), e1[p], zk); }
        Z[(0 * Q + o) * P2 + col] = zm;
        Z[(1 * Q + o) * P2 + col] = zk;
      }
    }
    __syncthreads();

    // ---- 2. x contraction: A = M_x Zm, E = K_x Zm + M_x Zk  (lines (oz, y)) ----
    if (lane < Q * P) {
      const int oz = lane / P, y = lane % P;
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
          av = fma(band_m(a.band, j, x), zm[x], av);
          ev = fma(band_k(a.band, j, x), zm[x], ev);
          ev = fma(band_m(a.band, j, x), zk[x], ev);
        }
        AE[((0 * Q + oz) * P + y) * Q + o] = av;
        AE[((1 * Q + oz) * P + y) * Q + o] = ev;
      }
    }
    __syncthreads();

    // ---- 3. y contraction, local residual, T^T along y  (lines (oz, ox)) ----
    if (lane < Q2) {
      const int oz = ly, ox = lx;
      T av[P], ev[P];
#pragma unroll
      for (int y = 0; y < P; ++y) {
        av[y] = AE[((0 * Q + oz) * P + y) * Q + ox];
        ev[y] = AE[((1 * Q + oz) * P + y) * Q + ox];
      }
      T r[Q], m[Q];
#pragma unroll
      for (int o = 0; o < Q; ++o) {
        const int j = o + 1;
        T acc = T(0);
#pragma unroll
        for (int y = 0; y < P; ++y) {
          if (y < band_lo(j, K) || y > band_hi(j, K)) continue;
          acc = fma(band_k(a.band, j, y), av[y], acc);
          acc = fma(band_m(a.band, j, y), ev[y], acc);
        }
        r[o] = bv[p][o] - acc;
      }
      fdm_forward<T, K>(a.f, r, m);
#pragma unroll
      for (int jm = 0; jm < Q; ++jm) W0[(oz * Q + jm) * Q + ox] = m[jm];
    }
    __syncthreads();

    // ---- 4. T^T along x  (lines (oz, my)) ----
    if (lane < Q2) {
      T v[Q], m[Q];
#pragma unroll
      for (int x = 0; x < Q; ++x) v[x] = W0[lane * Q + x];
      fdm_forward<T, K>(a.f, v, m);
#pragma unroll
      for (int jm = 0; jm < Q; ++jm) W1[lane * Q + jm] = m[jm];
    }
    __syncthreads();

    // ---- 5. T^T along z and 1/Lambda  (lines (my, mx)) ----
    if (lane < Q2) {
      const int my = ly, mx = lx;
      T v[Q], c[Q];
#pragma unroll
      for (int z = 0; z < Q; ++z) v[z] = W1[z * Q2 + lane];
      fdm_forward<T, K>(a.f, v, c);
      T lmy = a.lam[0], lmx = a.lam[0];
#pragma unroll
      for (int q = 1; q < Q; ++q) {
        lmy = (my == q) ? a.lam[q] : lmy;
        lmx = (mx == q) ? a.lam[q] : lmx;
      }
      const T s2 = lmy + lmx;
#pragma unroll
      for (int jm = 0; jm < Q; ++jm) {
        W0[jm * Q2 + lane] = c[jm] * inv_eig(s2 + a.lam[jm]);
      }
    }
    __syncthreads();

    // ---- 6. T along x  (lines (mz, my)) ----
    if (lane < Q2) {
      T c[Q], d[Q];
#pragma unroll
      for (int jm = 0; jm < Q; ++jm) c[jm] = W0[lane * Q + jm];
      fdm_backward<T, K>(a.f, c, d);
#pragma unroll
      for (int x = 0; x < Q; ++x) W1[lane * Q + x] = d[x];
    }
    __syncthreads();

    // ---- 7. T along y  (lines (mz, x)) ----
    if (lane < Q2) {
      const int mz = ly, x = lx;
      T c[Q], d[Q];
#pragma unroll
      for (int jm = 0; jm < Q; ++jm) c[jm] = W1[(mz * Q + jm) * Q + x];
      fdm_backward<T, K>(a.f, c, d);
#pragma unroll
      for (int y = 0; y < Q; ++y) W0[(mz * Q + y) * Q + x] = d[y];
    }
    __syncthreads();

    // ---- 8. T along z, store the new interior plane by plane  (lines (y, x)) ----
    if (lane < Q2) {
      T c[Q], d[Q];
#pragma unroll
      for (int jm = 0; jm < Q; ++jm) c[jm] = W0[jm * Q2 + lane];
      fdm_backward<T, K>(a.f, c, d);
      const unsigned off = srow * (unsigned)(1 + ly) + (unsigned)(1 + lx + x0) * (unsigned)sizeof(T);
#pragma unroll
      for (int z = 0; z < Q; ++z) buf_store<T>(d[z], ur, off, sbase + splane * (z + 1));
    }
  }
}

}  // namespace vps
