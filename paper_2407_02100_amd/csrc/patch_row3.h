// Patch smoother kernel for 3D, constant coefficient: a row of x-adjacent
// patches of one color per wavefront, lanes on node columns.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "patch_wave.h"

namespace vps {

// ---------------------------------------------------------------------------
// Same update as patch_wave3_kernel (exact local solve from the closure with
// the interior values taken as zero, fast diagonalisation in even/odd form).
// Same-color patches 2 vertices apart along x share a closure face, so G of
// them side by side span G*2K + 1 node columns.  One lane per column loads
// the closure rows of the G patches that lie on the rim of the (y, z)
// cross-section (y or z on the closure boundary) as contiguous runs of up to
// 61 values; the rows that cross the patches' interiors carry nonzero values
// only in the G + 1 x-face columns: at K = 4 a prepass handles those apart
// (which takes 45 registers off every lane), at K = 2, 3 the face lanes load
// them with the rim and the other lanes hold zeros.  Per patch
// this touches about a third of the cache lines of the one-patch kernel,
// whose short rows 2 KiB apart bind it to the per-CU vector-memory path.
//
// Stages of the wave that owns G patches:
//   P. (K = 4) lanes = (x face, y): the interior (y, z) block of each x-face
//      column, contracted along z in registers and along y after an LDS
//      transpose, into its share of F_M and F_E (below), kept in LDS;
// then for each interior node plane oz of the patches in turn:
//   A. lanes = closure columns: z then y contraction of the rim of the
//      lane's column (held in registers) into the two x-line inputs of the
//      residual, F_M = (M_y M_z) u and F_E = (K_y M_z + M_y K_z) u, and the
//      right-hand side rows of the plane, into LDS;
//   B. lanes = (patch, oy): x contraction of the row from LDS (the face
//      columns with their interior share added), local residual, T^T along
//      x, kept in registers;
// then, with every plane done,
//   C. T^T along z in registers; LDS transpose to lanes (patch, mx): T^T
//      along y, 1/Lambda, T along y, T along z, all in registers;
//   D. lanes (patch, y): T along x on their x lines in LDS, in place; then
//      lanes (patch, interior column) store the new interior as x rows.

template <int K>
struct Row3Shape {
  static constexpr int P = 2 * K + 1, Q = 2 * K - 1, S = 2 * K;
  static constexpr int G = 63 / S;     // patches per wave
  static constexpr int C = G * S + 1;  // closure columns of the G patches
  static constexpr int GQ = G * Q;     // interior columns (and x rows) of the G patches
  static constexpr int F = G + 1;                 // x-face columns of the G patches
  static constexpr bool FACE_PASS = K >= 4;        // stage P (measured faster at K = 4 only)
  static constexpr int PLANE = 3 * Q * C;          // LDS of stages A-B: F_M, F_E, rhs rows of one plane
  static constexpr int FACE = FACE_PASS ? 2 * Q * Q * F : 0;  // LDS of stages P-B: the faces' interior share
  static constexpr int CUBE = G * Q * Q * Q;       // LDS of stages C-D: the G interiors
  static constexpr int LDS = PLANE + FACE > CUBE ? PLANE + FACE : CUBE;
  static_assert(C <= 64 && GQ <= 64 && F * Q <= 64, "a row of patches must fit one wave");
  static_assert(FACE <= PLANE, "the prepass transpose (FACE values at the start) stays below the face buffer");
};

template <typename T, int K>
struct Row3Args {
  T* __restrict__ u;
  const T* __restrict__ b;
  int n1;
  int v0[3];
  int np[3];
  int ngx;             // groups of G patches per color row: ceil(np[0] / G)
  unsigned ngroups;    // ngx * np[1] * np[2]
  unsigned vec_bytes;  // bytes of one level vector (< 2^32)
  unsigned magic_g, magic_y;  // magic_of(ngx), magic_of(np[1]) (see div_magic)
  SymBand<T, K> band;  // interior rows of the 2-cell patch mass and stiffness matrices
  WaveFdm<T, K> f;
  T lam[2 * K - 1];  // 1D generalized eigenvalues in the internal mode order
};

template <typename T, int K>
__global__ void __launch_bounds__(64) patch_row3_kernel(const Row3Args<T, K> a) {
  using R = Row3Shape<K>;
  constexpr int P = R::P, Q = R::Q, S = R::S, G = R::G, C = R::C, GQ = R::GQ, M = K - 1;
  constexpr int F = R::F;
  __shared__ T L[R::LDS];
  T* FM = L;              // [oy][column] of the current plane
  T* FE = L + Q * C;      // [oy][column]
  T* BB = L + 2 * Q * C;  // [oy][column]: right-hand side of the current plane
  T* DM = L + R::PLANE;   // [oz][oy][face]: interior share of F_M at the x-face columns
  T* DE = DM + Q * Q * F; // [oz][oy][face]: ... of F_E
  T* ZI = L;              // stage P: [t][face][oz][y] after the z contraction (below the face buffer)
  T* W = L;               // stages C-D: [patch][.][.][.]

  const unsigned h = blockIdx.x;
  const unsigned per = gridDim.x / kXcd;
  const unsigned g = (h % kXcd) * per + h / kXcd;  // one contiguous slab of groups per XCD
  if (g >= a.ngroups) return;
  const int lane = threadIdx.x;
  const unsigned ngx = (unsigned)a.ngx, npy = (unsigned)a.np[1];
  const unsigned q1 = div_magic(g, ngx, a.magic_g);
  const unsigned q2 = div_magic(q1, npy, a.magic_y);
  const int px0 = G * (int)(g - q1 * ngx);
  const int py = (int)(q1 - q2 * npy);
  const int pz = (int)q2;
  const int nact = min(G, a.np[0] - px0);  // patches of the group that exist
  const int cmax = nact * S;               // last closure column that exists
  const unsigned n1 = (unsigned)a.n1;
  const size_t n2 = (size_t)n1 * n1;
  const size_t base = (size_t)(K * (a.v0[0] + 2 * px0 - 1)) + (size_t)n1 * (size_t)(K * (a.v0[1] + 2 * py - 1)) +
                      n2 * (size_t)(K * (a.v0[2] + 2 * pz - 1));
  const __amdgpu_buffer_rsrc_t ur = make_rsrc(a.u, a.vec_bytes);
  const __amdgpu_buffer_rsrc_t br = make_rsrc(a.b, a.vec_bytes);
  const unsigned sbase = (unsigned)(base * sizeof(T));  // group origin, bytes
  const unsigned srow = n1 * (unsigned)sizeof(T);
  const unsigned splane = (unsigned)(n2 * sizeof(T));

  // ---- every load of u, issued before any arithmetic: the rim rows of the
  //      closures (lanes = columns; lanes past the group repeat its last
  //      column) and the interior rows of the x-face columns (K = 4: lanes =
  //      (face, y), faces past the group repeat its last face; else the face
  //      lanes, the other lanes holding zeros) ----
  constexpr bool FP = R::FACE_PASS;
  const unsigned offc = (unsigned)min(lane, cmax) * (unsigned)sizeof(T);
  const bool face = (lane % S) == 0 && lane <= cmax;
  T uc[P][P];  // [z][y] of the lane's column (K = 4: rim only)
#pragma unroll
  for (int z = 0; z < P; ++z)
#pragma unroll
    for (int y = 0; y < P; ++y) {
      if (y == 0 || y == P - 1 || z == 0 || z == P - 1) uc[z][y] = buf_load<T>(ur, offc, sbase + splane * z + srow * y);
      else if constexpr (!FP) uc[z][y] = face ? buf_load<T>(ur, offc, sbase + splane * z + srow * y) : T(0);
    }
  const int lf = min(lane, F * Q - 1);
  const int ff = lf / Q, fy = lf % Q;  // (face, interior row) of stage P
  const unsigned offf = (unsigned)min(ff * S, cmax) * (unsigned)sizeof(T) + srow * (unsigned)(fy + 1);
  T uf[Q];  // the face column's interior rows at y = fy + 1, along z
  if constexpr (FP) {
#pragma unroll
    for (int z = 0; z < Q; ++z) uf[z] = buf_load<T>(ur, offf, sbase + splane * (z + 1));
  }
  T bnext[Q];  // right-hand side rows of the next plane (lanes = columns)
#pragma unroll
  for (int y = 0; y < Q; ++y) bnext[y] = buf_load<T>(br, offc, sbase + splane + srow * (y + 1));

  // ---- P. the x faces' interior blocks: z contraction (lanes (face, y)),
  //      y contraction (lanes (face, oz)) into DM, DE ----
  if (FP && lane < F * Q) {
#pragma unroll
    for (int oz = 0; oz < Q; ++oz) {
      const int jz = oz + 1;
      T sm = T(0), sk = T(0);
#pragma unroll
      for (int z = 1; z < P - 1; ++z) {
        if (z < band_lo(jz, K) || z > band_hi(jz, K)) continue;
        sm = fma(sym_m(a.band, jz, z), uf[z - 1], sm);
        sk = fma(sym_k(a.band, jz, z), uf[z - 1], sk);
      }
      ZI[(ff * Q + oz) * Q + fy] = sm;
      ZI[((F + ff) * Q + oz) * Q + fy] = sk;
    }
  }
  if constexpr (FP) __syncthreads();
  if (FP && lane < F * Q) {
    const int oz = fy;
    T zm[Q], zk[Q];
#pragma unroll
    for (int y = 0; y < Q; ++y) {
      zm[y] = ZI[(ff * Q + oz) * Q + y];
      zk[y] = ZI[((F + ff) * Q + oz) * Q + y];
    }
#pragma unroll
    for (int oy = 0; oy < Q; ++oy) {
      const int jy = oy + 1;
      T fm = T(0), fe = T(0);
#pragma unroll
      for (int y = 1; y < P - 1; ++y) {
        if (y < band_lo(jy, K) || y > band_hi(jy, K)) continue;
        fm = fma(sym_m(a.band, jy, y), zm[y - 1], fm);
        fe = fma(sym_k(a.band, jy, y), zm[y - 1], fe);
        fe = fma(sym_m(a.band, jy, y), zk[y - 1], fe);
      }
      DM[(oz * Q + oy) * F + ff] = fm;
      DE[(oz * Q + oy) * F + ff] = fe;
    }
  }
  if constexpr (FP) __syncthreads();  // the planes of stage A overwrite ZI

  const int l2 = min(lane, GQ - 1);
  const int pp = l2 / Q, ll = l2 % Q;  // (patch, line) of stages B-D
  const int c0 = pp * S;               // the patch's first closure column
  T mr[Q][Q];                          // stage B output of lane (pp, oy = ll): [oz][mx]

#pragma unroll
  for (int oz = 0; oz < Q; ++oz) {
    const int jz = oz + 1;
    T bcur[Q];
#pragma unroll
    for (int y = 0; y < Q; ++y) bcur[y] = bnext[y];
    if (oz + 1 < Q) {
#pragma unroll
      for (int y = 0; y < Q; ++y) bnext[y] = buf_load<T>(br, offc, sbase + splane * (oz + 2) + srow * (y + 1));
    }
    // ---- A. lanes = columns: z then y contraction of plane oz ----
    if (lane < C) {
      T zm[P], zk[P];
#pragma unroll
      for (int y = 0; y < P; ++y) {
        T sm = T(0), sk = T(0);
#pragma unroll
        for (int z = 0; z < P; ++z) {
          if (z < band_lo(jz, K) || z > band_hi(jz, K)) continue;
          if (FP && y > 0 && y < P - 1 && z > 0 && z < P - 1) continue;  // off the rim (stage P)
          sm = fma(sym_m(a.band, jz, z), uc[z][y], sm);
          sk = fma(sym_k(a.band, jz, z), uc[z][y], sk);
        }
        zm[y] = sm;
        zk[y] = sk;
      }
#pragma unroll
      for (int oy = 0; oy < Q; ++oy) {
        const int jy = oy + 1;
        T fm = T(0), fe = T(0);
#pragma unroll
        for (int y = 0; y < P; ++y) {
          if (y < band_lo(jy, K) || y > band_hi(jy, K)) continue;
          fm = fma(sym_m(a.band, jy, y), zm[y], fm);
          fe = fma(sym_k(a.band, jy, y), zm[y], fe);
          fe = fma(sym_m(a.band, jy, y), zk[y], fe);
        }
        FM[oy * C + lane] = fm;
        FE[oy * C + lane] = fe;
        BB[oy * C + lane] = bcur[oy];
      }
    }
    __syncthreads();
    // ---- B. lanes = (patch, oy): x contraction, local residual, T^T along x ----
    if (lane < GQ) {
      const int oy = ll;
      T fm[P], fe[P], r[Q];
#pragma unroll
      for (int x = 0; x < P; ++x) {
        fm[x] = FM[oy * C + c0 + x];
        fe[x] = FE[oy * C + c0 + x];
      }
      if constexpr (FP) {
        fm[0] += DM[(oz * Q + oy) * F + pp];
        fe[0] += DE[(oz * Q + oy) * F + pp];
        fm[P - 1] += DM[(oz * Q + oy) * F + pp + 1];
        fe[P - 1] += DE[(oz * Q + oy) * F + pp + 1];
      }
#pragma unroll
      for (int ox = 0; ox < Q; ++ox) {
        const int jx = ox + 1;
        T s = T(0);
#pragma unroll
        for (int x = 0; x < P; ++x) {
          if (x < band_lo(jx, K) || x > band_hi(jx, K)) continue;
          s = fma(sym_k(a.band, jx, x), fm[x], s);
          s = fma(sym_m(a.band, jx, x), fe[x], s);
        }
        r[ox] = BB[oy * C + c0 + 1 + ox] - s;
      }
      fdm_forward<T, K>(a.f, r, mr[oz]);
    }
    __syncthreads();  // the next plane overwrites FM, FE, BB
  }

  // ---- C. T^T along z (registers), then lanes (patch, mx) ----
  if (lane < GQ) {
    const int oy = ll;
#pragma unroll
    for (int mx = 0; mx < Q; ++mx) {
      T v[Q], c[Q];
#pragma unroll
      for (int oz = 0; oz < Q; ++oz) v[oz] = mr[oz][mx];
      fdm_forward<T, K>(a.f, v, c);
#pragma unroll
      for (int mz = 0; mz < Q; ++mz) W[((pp * Q + mx) * Q + mz) * Q + oy] = c[mz];
    }
  }
  __syncthreads();
  T e[Q][Q];  // lane (pp, mx = ll): [mz][y], then [z][y]
  if (lane < GQ) {
    const int mx = ll;
    T lmx = a.lam[0];
#pragma unroll
    for (int q = 1; q < Q; ++q) lmx = (mx == q) ? a.lam[q] : lmx;
#pragma unroll
    for (int mz = 0; mz < Q; ++mz) {
      T v[Q], c[Q];
#pragma unroll
      for (int oy = 0; oy < Q; ++oy) v[oy] = W[((pp * Q + mx) * Q + mz) * Q + oy];
      fdm_forward<T, K>(a.f, v, c);  // T^T along y
      const T s2 = lmx + a.lam[mz];
#pragma unroll
      for (int my = 0; my < Q; ++my) {
        if constexpr (sizeof(T) == 4) c[my] *= __builtin_amdgcn_rcpf(s2 + a.lam[my]);
        else c[my] /= (s2 + a.lam[my]);
      }
      fdm_backward<T, K>(a.f, c, e[mz]);  // T along y
    }
#pragma unroll
    for (int y = 0; y < Q; ++y) {  // T along z
      T v[Q], d[Q];
#pragma unroll
      for (int mz = 0; mz < Q; ++mz) v[mz] = e[mz][y];
      fdm_backward<T, K>(a.f, v, d);
#pragma unroll
      for (int z = 0; z < Q; ++z) e[z][y] = d[z];
    }
  }
  __syncthreads();  // every lane has read W
  if (lane < GQ) {
    const int mx = ll;
#pragma unroll
    for (int z = 0; z < Q; ++z)
#pragma unroll
      for (int y = 0; y < Q; ++y) W[((pp * Q + z) * Q + y) * Q + mx] = e[z][y];
  }
  __syncthreads();

  // ---- D. lanes = (patch, y): T along x on the lane's own x lines, in place;
  //      then lanes = (patch, interior column x): store the x rows ----
  if (lane < GQ) {
    const int y = ll;
#pragma unroll
    for (int z = 0; z < Q; ++z) {
      T* w = W + ((pp * Q + z) * Q + y) * Q;
      T c[Q], d[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) c[q] = w[q];
      fdm_backward<T, K>(a.f, c, d);
#pragma unroll
      for (int x = 0; x < Q; ++x) w[x] = d[x];
    }
  }
  __syncthreads();
  if (lane < GQ && pp < nact) {
    const int x = ll;
    const unsigned off2 = (unsigned)(c0 + 1 + x) * (unsigned)sizeof(T);
#pragma unroll
    for (int z = 0; z < Q; ++z)
#pragma unroll
      for (int y = 0; y < Q; ++y)
        buf_store<T>(W[((pp * Q + z) * Q + y) * Q + x], ur, off2, sbase + splane * (z + 1) + srow * (y + 1));
  }
}

}  // namespace vps
