// Patch smoother kernel for 3D, constant coefficient, degree 5: a row of
// x-adjacent patches of one color per workgroup of two wavefronts.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "patch_row3.h"
#include "patch_wave.h"

namespace vps {

// ---------------------------------------------------------------------------
// The update of patch_row3_kernel (exact local solve from the closure with the
// interior values taken as zero, fast diagonalisation in even/odd form) for
// K = 5, where one wave cannot hold both what a closure column needs over the
// planes (its ring of 4K values) and what a (patch, row) lane accumulates over
// the planes ((2K-1)^2 values): at FP64 that is 40 + 81 doubles per lane.  So
// the two roles go to two waves of one workgroup, which work on different
// planes at the same time through double-buffered plane arrays:
//
//   wave 0 (lanes = closure columns of the G patches): loads the ring of its
//     column and the right-hand side rows; per interior plane oz: z then y
//     contraction of its column into F_M = (M_y M_z) u and
//     F_E = (K_y M_z + M_y K_z) u (rows oy) and the right-hand side rows,
//     into plane buffer oz mod 2;
//   wave 1: first the x faces' interior blocks (lanes (face, y): z
//     contraction, LDS transpose, lanes (face, oz): y contraction) into their
//     share of F_M, F_E; then per plane, one plane behind wave 0, lanes
//     (patch, oy): x contraction, local residual, T^T along x, kept in
//     registers over the planes;
//   wave 1, after the last plane: T^T along z into the interior cube;
//   both waves: the y transforms and 1/Lambda, T along z, T along x, each pass
//     over all lines of its direction spread over the 128 lanes (the values
//     stay in LDS between the passes, so that no lane holds a whole patch
//     slab), then the stores, the (z, y) rows alternating between the waves.
//
// FP64 keeps the first two planes of wave 1's accumulated rows in LDS, so that
// both programs fit the registers of two waves per SIMD.
//
// Groups of G consecutive patches of the color as in patch_row3_kernel (packed
// along the rows of patches when a row holds at least G patches).

template <int K>
struct Row5Shape {
  static constexpr int P = 2 * K + 1, Q = 2 * K - 1, S = 2 * K;
  // patches per workgroup: G*S + 2 columns, G + 2 faces of Q rows and G Q lines fit one wave
  static constexpr int G = ((64 - 2) / S < 64 / Q - 2) ? (64 - 2) / S : 64 / Q - 2;
  static constexpr int C = G * S + 2;     // closure columns (a packed group: two runs)
  static constexpr int CS = C | 1;        // LDS row stride of the plane buffers (odd: bank spread)
  static constexpr int GQ = G * Q;        // (patch, line) lanes
  static constexpr int F = G + 2;         // x faces
  static constexpr int PL = 3 * Q * CS;   // one plane buffer: F_M, F_E, right-hand side rows
  static constexpr int FACE = 2 * Q * Q * F;  // the faces' interior share of F_M and F_E
  static constexpr int PS = Q * Q * Q + 1;    // patch stride of the interior cube
  static constexpr int CUBE = G * PS;
  // leading planes of the (patch, row) lanes' accumulated rows kept in LDS rather than in registers
  // (FP64: so that a lane stays within the registers of two waves per SIMD)
  template <typename T>
  static constexpr int MRL = sizeof(T) == 8 ? 2 : 0;
  template <typename T>
  static constexpr int LDS = (2 * PL + FACE + MRL<T> * Q * GQ > CUBE) ? 2 * PL + FACE + MRL<T> * Q * GQ : CUBE;
  static_assert(C <= 64 && GQ <= 64 && F * Q <= 64, "a row of patches must fit one wave");
  static_assert(FACE <= PL, "the prepass transpose lives in the second plane buffer");
};

template <typename T, int K>
struct Row5Fdm {
  WaveFdm<T, K> f;
  T lam[2 * K - 1];
};

// Rows (z, y) of one interior x column with z*Q + y = PAR mod 2, from its [z][y] slab of the cube.
template <typename T, int Q, int PAR>
__device__ inline void row5_store_rows(const T* wx, __amdgpu_buffer_rsrc_t ur, unsigned off, unsigned sbase,
                                       unsigned splane, unsigned srow) {
#pragma unroll
  for (int zy = PAR; zy < Q * Q; zy += 2) {
    const int z = zy / Q, y = zy - z * Q;
    buf_store<T>(wx[zy], ur, off, sbase + splane * (z + 1) + srow * (y + 1));
  }
}

template <typename T, int K>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 2 : 4)))
patch_row5_kernel(const Row3Args<T, K> a) {
  using R = Row5Shape<K>;
  constexpr int P = R::P, Q = R::Q, S = R::S, G = R::G, C = R::C, CS = R::CS, F = R::F, GQ = R::GQ;
  constexpr int PL = R::PL, PS = R::PS, MRL = R::template MRL<T>;
  __shared__ T L[R::template LDS<T>];
  __shared__ Row5Fdm<T, K> FS;  // FDM factors and eigenvalues (in LDS: not enough scalar registers)
  T* DM = L + 2 * PL;           // [oz][oy][face]: interior share of F_M at the x-face columns
  T* DE = DM + Q * Q * F;       // [oz][oy][face]: ... of F_E
  T* ZI = L + PL;               // prepass transpose [t][face][oz][y], in plane buffer 1 (free until then)
  T* MR = DE + Q * Q * F;       // [oz][mx][lane]: planes oz < MRL of the accumulated rows
  T* W = L;                     // after the planes: the G interiors, PS values apart

  const unsigned h = blockIdx.x;
  const unsigned per = gridDim.x / kXcd;
  const unsigned g = (h % kXcd) * per + h / kXcd;  // one contiguous slab of groups per XCD
  if (g >= a.ngroups) return;
  const int tid = threadIdx.x;
  const int wv = tid >> 6;  // 0: columns, 1: (patch, row) lanes
  const int lane = tid & 63;
  if (tid < K * K) FS.f.Te[tid] = a.f.Te[tid];
  if (tid < (K - 1) * (K - 1)) FS.f.To[tid] = a.f.To[tid];
  if (tid < Q) FS.lam[tid] = a.lam[tid];

  const unsigned npx = (unsigned)a.np[0], npy = (unsigned)a.np[1];
  const unsigned n1 = (unsigned)a.n1;
  const size_t n2 = (size_t)n1 * n1;
  int px0, py, pz, nact, nrun1;
  unsigned run2 = 0;
  if (a.packed) {
    const unsigned t0 = (unsigned)G * g;
    const unsigned r = div_magic(t0, npx, a.magic_x);
    const unsigned q2 = div_magic(r, npy, a.magic_y);
    px0 = (int)(t0 - r * npx);
    py = (int)(r - q2 * npy);
    pz = (int)q2;
    nact = (int)min((unsigned)G, a.npatch - t0);
    nrun1 = min(nact, (int)npx - px0);
    if (nrun1 < nact) {
      const long long dy = (py + 1 < (int)npy) ? (long long)(2 * K) * n1
                                               : (long long)(2 * K) * (long long)n2 - (long long)(2 * K) * n1 * (npy - 1);
      run2 = (unsigned)((dy - (long long)(2 * K) * px0) * (long long)sizeof(T));
    }
  } else {
    const unsigned ngx = (unsigned)a.ngx;
    const unsigned q1 = div_magic(g, ngx, a.magic_g);
    const unsigned q2 = div_magic(q1, npy, a.magic_y);
    px0 = G * (int)(g - q1 * ngx);
    py = (int)(q1 - q2 * npy);
    pz = (int)q2;
    nact = min(G, (int)npx - px0);
    nrun1 = nact;
  }
  const int cs = nrun1 * S;
  const int cmax = nact * S + (nrun1 < nact ? 1 : 0);
  const size_t base = (size_t)(K * (a.v0[0] + 2 * px0 - 1)) + (size_t)n1 * (size_t)(K * (a.v0[1] + 2 * py - 1)) +
                      n2 * (size_t)(K * (a.v0[2] + 2 * pz - 1));
  auto colb = [&](int c) -> unsigned {
    return c <= cs ? (unsigned)c * (unsigned)sizeof(T) : run2 + (unsigned)(c - cs - 1) * (unsigned)sizeof(T);
  };
  const __amdgpu_buffer_rsrc_t ur = make_rsrc(a.u, a.vec_bytes);
  const __amdgpu_buffer_rsrc_t br = make_rsrc(a.b, a.vec_bytes);
  const unsigned sbase = (unsigned)(base * sizeof(T));
  const unsigned srow = n1 * (unsigned)sizeof(T);
  const unsigned splane = (unsigned)(n2 * sizeof(T));

  // The two waves run separate programs up to the cube (so that the column
  // ring and the accumulated rows never share registers); each passes the same
  // 11 workgroup barriers: 2 in the prologue, one per plane.
  if (wv == 0) {
    // ---- wave 0: the ring of the lane's column (lanes past the group repeat its
    //      last column) and the first right-hand side rows ----
    const unsigned offc = colb(min(lane, cmax));
    T uc[P][P];  // [z][y] of the lane's column, ring only (y or z on the closure boundary)
    T bnext[Q];  // right-hand side rows of the next plane
#pragma unroll
    for (int z = 0; z < P; ++z)
#pragma unroll
      for (int y = 0; y < P; ++y)
        if (y == 0 || y == P - 1 || z == 0 || z == P - 1) uc[z][y] = buf_load<T>(ur, offc, sbase + splane * z + srow * y);
#pragma unroll
    for (int y = 0; y < Q; ++y) bnext[y] = buf_load<T>(br, offc, sbase + splane + srow * (y + 1));
    // plane oz (jz = oz + 1) of F_M, F_E and the right-hand side rows into
    // plane buffer oz mod 2, one plane ahead of wave 1
#pragma unroll
    for (int oz = 0; oz < Q; ++oz) {
      const int jz = oz + 1;
      T* pb = L + (oz & 1) * PL;
      T bcur[Q];
#pragma unroll
      for (int y = 0; y < Q; ++y) bcur[y] = bnext[y];
      if (oz + 1 < Q) {
#pragma unroll
        for (int y = 0; y < Q; ++y) bnext[y] = buf_load<T>(br, offc, sbase + splane * (oz + 2) + srow * (y + 1));
      }
      if (lane < C) {
        T zm[P], zk[P];
#pragma unroll
        for (int y = 0; y < P; ++y) {
          T sm = T(0), sk = T(0);
#pragma unroll
          for (int z = 0; z < P; ++z) {
            if (z < band_lo(jz, K) || z > band_hi(jz, K)) continue;
            if (y > 0 && y < P - 1 && z > 0 && z < P - 1) continue;  // off the ring (the faces' prepass)
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
          pb[oy * CS + lane] = fm;
          pb[Q * CS + oy * CS + lane] = fe;
          pb[2 * Q * CS + oy * CS + lane] = bcur[oy];
        }
      }
      if (oz == 0) {
        __syncthreads();  // 1: plane 0 and the faces' z contraction are in LDS
        __syncthreads();  // 2: the faces' share is complete, plane buffer 1 free
      } else {
        __syncthreads();  // 2 + oz: plane oz written, plane oz - 1 read
      }
    }
    __syncthreads();  // 11: wave 1 has read plane Q - 1
  } else {
    // ---- wave 1: the interior rows of the x-face columns (lanes (face, y); faces
    //      past the group repeat its last face): z contraction into ZI ----
    const int lf = min(lane, F * Q - 1);
    const int ff = lf / Q, fy = lf % Q;
    const int nfaces = nact + 1 + (nrun1 < nact ? 1 : 0);
    const int fcl = min(ff, nfaces - 1);
    const unsigned offf = colb(fcl <= nrun1 ? fcl * S : (fcl - 1) * S + 1) + srow * (unsigned)(fy + 1);
    {
      T uf[Q];  // the face column's interior rows at y = fy + 1, along z
#pragma unroll
      for (int z = 0; z < Q; ++z) uf[z] = buf_load<T>(ur, offf, sbase + splane * (z + 1));
      if (lane < F * Q) {
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
    }
    __syncthreads();  // 1
    // the faces' y contraction into DM, DE (lanes (face, oz))
    if (lane < F * Q) {
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
    __syncthreads();  // 2: ZI (plane buffer 1) is free again; DM, DE complete
    // ---- per plane, one behind wave 0: lanes (patch, oy): x contraction, local
    //      residual, T^T along x, into registers ----
    const int l2 = min(lane, GQ - 1);
    const int pp = l2 / Q, oy = l2 % Q;
    const int pr2 = pp >= nrun1 ? 1 : 0;
    const int c0 = pp * S + pr2;
    const int fl = pp + pr2;
    T mr[Q][Q];  // [oz][mx] (planes oz < MRL in MR instead)
#pragma unroll
    for (int oz = 0; oz < Q; ++oz) {
      if (lane < GQ) {
        const T* pb = L + (oz & 1) * PL;
        // x contraction column by column (few values live next to mr)
        T r[Q];
#pragma unroll
        for (int ox = 0; ox < Q; ++ox) r[ox] = T(0);
#pragma unroll
        for (int x = 0; x < P; ++x) {
          T fmx = pb[oy * CS + c0 + x];
          T fex = pb[Q * CS + oy * CS + c0 + x];
          if (x == 0 || x == P - 1) {
            fmx += DM[(oz * Q + oy) * F + fl + (x == 0 ? 0 : 1)];
            fex += DE[(oz * Q + oy) * F + fl + (x == 0 ? 0 : 1)];
          }
#pragma unroll
          for (int ox = 0; ox < Q; ++ox) {
            const int jx = ox + 1;
            if (x < band_lo(jx, K) || x > band_hi(jx, K)) continue;
            r[ox] = fma(sym_k(a.band, jx, x), fmx, r[ox]);
            r[ox] = fma(sym_m(a.band, jx, x), fex, r[ox]);
          }
        }
#pragma unroll
        for (int ox = 0; ox < Q; ++ox) r[ox] = pb[2 * Q * CS + oy * CS + c0 + 1 + ox] - r[ox];
        if (oz < MRL) {
          T t[Q];
          fdm_forward<T, K>(FS.f, r, t);
#pragma unroll
          for (int mx = 0; mx < Q; ++mx) MR[(oz * Q + mx) * GQ + lane] = t[mx];
        } else {
          fdm_forward<T, K>(FS.f, r, mr[oz]);
        }
      }
      __syncthreads();  // 3 + oz
    }
    // ---- T^T along z (registers), then the cube (wave 0 is past its last plane) ----
    if (lane < GQ) {
#pragma unroll
      for (int mx = 0; mx < Q; ++mx) {
        T v[Q], c[Q];
#pragma unroll
        for (int oz = 0; oz < Q; ++oz) v[oz] = oz < MRL ? MR[(oz * Q + mx) * GQ + lane] : mr[oz][mx];
        fdm_forward<T, K>(FS.f, v, c);
#pragma unroll
        for (int mz = 0; mz < Q; ++mz) W[pp * PS + (mx * Q + mz) * Q + oy] = c[mz];
      }
    }
  }
  __syncthreads();  // both waves: the cube holds T^T_z T^T_x of the residuals
  // The remaining line transforms, each pass over the G*Q*Q lines of one direction spread over the
  // workgroup's 128 lanes (the cube is [x][z][y] per patch, PS values apart).
  constexpr int NL = G * Q * Q;
  constexpr int IT = (NL + 127) / 128;
  // T^T along y, 1/Lambda, T along y: lines (p, mx, mz), contiguous
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int t = it * 128 + tid;
    if (t < NL) {
      const int p = t / (Q * Q), r = t - p * (Q * Q), mx = r / Q, mz = r - mx * Q;
      T* w = W + p * PS + r * Q;
      T v[Q], c[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) v[q] = w[q];
      fdm_forward<T, K>(FS.f, v, c);
      const T s2 = FS.lam[mx] + FS.lam[mz];
#pragma unroll
      for (int my = 0; my < Q; ++my) c[my] *= inv_eig(s2 + FS.lam[my]);
      fdm_backward<T, K>(FS.f, c, v);
#pragma unroll
      for (int q = 0; q < Q; ++q) w[q] = v[q];
    }
  }
  __syncthreads();
  // T along z: lines (p, mx, y), stride Q
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int t = it * 128 + tid;
    if (t < NL) {
      const int p = t / (Q * Q), r = t - p * (Q * Q), mx = r / Q, y = r - mx * Q;
      T* w = W + p * PS + mx * Q * Q + y;
      T v[Q], d[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) v[q] = w[q * Q];
      fdm_backward<T, K>(FS.f, v, d);
#pragma unroll
      for (int q = 0; q < Q; ++q) w[q * Q] = d[q];
    }
  }
  __syncthreads();
  // T along x: lines (p, z, y), stride Q*Q
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int t = it * 128 + tid;
    if (t < NL) {
      const int p = t / (Q * Q), r = t - p * (Q * Q);
      T* w = W + p * PS + r;
      T v[Q], d[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) v[q] = w[q * Q * Q];
      fdm_backward<T, K>(FS.f, v, d);
#pragma unroll
      for (int q = 0; q < Q; ++q) w[q * Q * Q] = d[q];
    }
  }
  __syncthreads();
  // store the new interiors as x rows: lanes (patch, interior column x), the (z, y) rows alternating
  // between the two waves
  if (lane < GQ) {
    const int p = lane / Q, x = lane - p * Q;
    if (p < nact) {
      const int qc0 = p * S + (p >= nrun1 ? 1 : 0);
      const unsigned off2 = colb(qc0 + 1 + x);
      const T* wx = W + p * PS + x * Q * Q;
      if (__builtin_amdgcn_readfirstlane(wv) == 0)
        row5_store_rows<T, Q, 0>(wx, ur, off2, sbase, splane, srow);
      else
        row5_store_rows<T, Q, 1>(wx, ur, off2, sbase, splane, srow);
    }
  }
}

}  // namespace vps
