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
// Groups: the patches of a color in lexicographic order (x fastest) are cut
// into groups of G consecutive patches, so that a row of 64 patches does not
// leave a group of one (which costs a whole wave); a group that reaches the
// end of a row of patches continues at the start of the next row, as a
// second run of columns with its own origin (G*2K + 2 columns in all).  Rows
// shorter than G patches keep one group per row piece.
//
// Stages of the wave that owns G patches:
//   P. (K = 4) lanes = (x face, y): the interior (y, z) block of each x-face
//      column, contracted along z in registers and along y after an LDS
//      transpose, into its share of F_M and F_E (below), kept in LDS;
// then for each interior node plane oz of the patches in turn:
//   A. lanes = closure columns: z then y contraction of the rim of the
//      lane's column (held in registers) into the two x-line inputs of the
//      residual, F_M = (M_y M_z) u and F_E = (K_y M_z + M_y K_z) u, and the
//      right-hand side rows of the plane, into LDS (K = 4: the column is only
//      the ring y or z in {0, P-1}, so F is a sum of four outer products of a
//      1D band column with the y sums of the z = 0, P-1 rows, taken once
//      before the planes, and the z sums of the y = 0, P-1 rows);
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
  // closure columns of the G patches: G*S + 1 when they lie in one row of
  // patches, one more when a packed group continues on the next row
  static constexpr int C = G * S + 2;
  static constexpr int GQ = G * Q;     // interior columns (and x rows) of the G patches
  static constexpr int F = G + 2;                 // x-face columns of the G patches (as C)
  static constexpr bool FACE_PASS = K >= 4;        // stage P (measured faster at K = 4 only)
  // LDS row stride of the plane buffers: odd, so that lanes (patch, oy) reading
  // column c0 + x of row oy (c0 = 2K patch) fall into different banks
  static constexpr int CS = C | 1;
  static constexpr int PLANE = 3 * Q * CS;         // LDS of stages A-B: F_M, F_E, rhs rows of one plane
  static constexpr int FACE = FACE_PASS ? 2 * Q * Q * F : 0;  // LDS of stages P-B: the faces' interior share
  // LDS of stages C-D: the G interiors, one patch every PS values (one more than
  // Q^3, which spreads the lanes (patch, line) of the line-wise passes over the banks)
  static constexpr int PS = Q * Q * Q + 1;
  static constexpr int CUBE = G * PS;
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
  int ngx;             // row groups: groups of G patches per color row, ceil(np[0] / G)
  int packed;          // 1: group g holds the patches G g .. G g + G - 1 of the color in
                       // lexicographic order (a group may continue on the next row of
                       // patches; needs np[0] >= G); 0: row groups
  unsigned ngroups;    // packed: ceil(np[0] np[1] np[2] / G); else ngx * np[1] * np[2]
  unsigned npatch;     // np[0] * np[1] * np[2]
  unsigned vec_bytes;  // bytes of one level vector (< 2^32)
  unsigned magic_g, magic_x, magic_y;  // magic_of(ngx), magic_of(np[0]), magic_of(np[1]) (see div_magic)
  SymBand<T, K> band;  // interior rows of the 2-cell patch mass and stiffness matrices
  WaveFdm<T, K> f;
  T lam[2 * K - 1];  // 1D generalized eigenvalues in the internal mode order
};

template <typename T, int K>
__global__ void __launch_bounds__(64) patch_row3_kernel(const Row3Args<T, K> a) {
  using R = Row3Shape<K>;
  constexpr int P = R::P, Q = R::Q, S = R::S, G = R::G, C = R::C, CS = R::CS, PS = R::PS, GQ = R::GQ, M = K - 1;
  constexpr int F = R::F;
  __shared__ T L[R::LDS];
  T* FM = L;              // [oy][column] of the current plane
  T* FE = L + Q * CS;     // [oy][column]
  T* BB = L + 2 * Q * CS; // [oy][column]: right-hand side of the current plane
  T* DM = L + R::PLANE;   // [oz][oy][face]: interior share of F_M at the x-face columns
  T* DE = DM + Q * Q * F; // [oz][oy][face]: ... of F_E
  T* ZI = L;              // stage P: [t][face][oz][y] after the z contraction (below the face buffer)
  T* W = L;               // stages C-D: [patch][.][.][.]

  const unsigned h = blockIdx.x;
  const unsigned per = gridDim.x / kXcd;
  const unsigned g = (h % kXcd) * per + h / kXcd;  // one contiguous slab of groups per XCD
  if (g >= a.ngroups) return;
  const int lane = threadIdx.x;
  const unsigned npx = (unsigned)a.np[0], npy = (unsigned)a.np[1];
  const unsigned n1 = (unsigned)a.n1;
  const size_t n2 = (size_t)n1 * n1;
  int px0, py, pz, nact;  // first patch of the group, patches that exist
  int nrun1;              // patches of the first run (the rest continue on the next row)
  unsigned run2 = 0;      // bytes from the group origin to the origin of the second run
  if (a.packed) {
    const unsigned t0 = (unsigned)G * g;
    const unsigned r = div_magic(t0, npx, a.magic_x);  // row of patches (py + np[1] pz)
    const unsigned q2 = div_magic(r, npy, a.magic_y);
    px0 = (int)(t0 - r * npx);
    py = (int)(r - q2 * npy);
    pz = (int)q2;
    nact = (int)min((unsigned)G, a.npatch - t0);
    nrun1 = min(nact, (int)npx - px0);
    if (nrun1 < nact) {
      // the next row starts at px = 0, one patch row up in y (or at y = 0 one up in z)
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
  const int cs = nrun1 * S;                          // last closure column of the first run
  const int cmax = nact * S + (nrun1 < nact ? 1 : 0);  // last closure column that exists
  const size_t base = (size_t)(K * (a.v0[0] + 2 * px0 - 1)) + (size_t)n1 * (size_t)(K * (a.v0[1] + 2 * py - 1)) +
                      n2 * (size_t)(K * (a.v0[2] + 2 * pz - 1));
  // byte offset of closure column c from the group origin (column cs + 1 starts the second run)
  auto colb = [&](int c) -> unsigned {
    return c <= cs ? (unsigned)c * (unsigned)sizeof(T) : run2 + (unsigned)(c - cs - 1) * (unsigned)sizeof(T);
  };
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
  const unsigned offc = colb(min(lane, cmax));
  const bool face = lane <= cmax && (lane <= cs ? lane % S == 0 : (lane - cs - 1) % S == 0);
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
  const int nfaces = nact + 1 + (nrun1 < nact ? 1 : 0);
  const int fcl = min(ff, nfaces - 1);  // faces past the group repeat its last face
  const unsigned offf = colb(fcl <= nrun1 ? fcl * S : (fcl - 1) * S + 1) + srow * (unsigned)(fy + 1);
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

  // K = 4: the column holds only the rim of the (y, z) square, so the y
  // contraction of its z = 0 and z = P-1 rows is done once for all planes:
  // F(jy, jz) = M_z(jz,0) a0(jy) + M_z(jz,P-1) a8(jy) + (y = 0, P-1 terms).
  // (FP32 only: in FP64 the 28 sums held over the planes would spill)
  constexpr bool RING = FP && sizeof(T) == 4;
  T ra0m[RING ? Q : 1], ra0k[RING ? Q : 1], ra8m[RING ? Q : 1], ra8k[RING ? Q : 1];
  if constexpr (RING) {
#pragma unroll
    for (int oy = 0; oy < Q; ++oy) {
      const int jy = oy + 1;
      T s0m = T(0), s0k = T(0), s8m = T(0), s8k = T(0);
#pragma unroll
      for (int y = 0; y < P; ++y) {
        if (y < band_lo(jy, K) || y > band_hi(jy, K)) continue;
        s0m = fma(sym_m(a.band, jy, y), uc[0][y], s0m);
        s0k = fma(sym_k(a.band, jy, y), uc[0][y], s0k);
        s8m = fma(sym_m(a.band, jy, y), uc[P - 1][y], s8m);
        s8k = fma(sym_k(a.band, jy, y), uc[P - 1][y], s8k);
      }
      ra0m[oy] = s0m;
      ra0k[oy] = s0k;
      ra8m[oy] = s8m;
      ra8k[oy] = s8k;
    }
  }

  const int l2 = min(lane, GQ - 1);
  const int pp = l2 / Q, ll = l2 % Q;  // (patch, line) of stages B-D
  const int pr2 = pp >= nrun1 ? 1 : 0;  // 1 if the patch is in the second run
  const int c0 = pp * S + pr2;          // the patch's first closure column
  const int fl = pp + pr2;              // the patch's first x face
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
      if constexpr (RING) {
        // rim-only column: the z = 0 and z = P-1 rows enter through the hoisted
        // y sums a0/a8, the y = 0 and y = P-1 rows (z inside) through c0/c8
        T c0m = T(0), c0k = T(0), c8m = T(0), c8k = T(0);
#pragma unroll
        for (int z = 1; z < P - 1; ++z) {
          if (z < band_lo(jz, K) || z > band_hi(jz, K)) continue;
          c0m = fma(sym_m(a.band, jz, z), uc[z][0], c0m);
          c0k = fma(sym_k(a.band, jz, z), uc[z][0], c0k);
          c8m = fma(sym_m(a.band, jz, z), uc[z][P - 1], c8m);
          c8k = fma(sym_k(a.band, jz, z), uc[z][P - 1], c8k);
        }
#pragma unroll
        for (int oy = 0; oy < Q; ++oy) {
          const int jy = oy + 1;
          T fm = T(0), fe = T(0);
          if (band_lo(jz, K) == 0) {
            fm = fma(sym_m(a.band, jz, 0), ra0m[oy], fm);
            fe = fma(sym_k(a.band, jz, 0), ra0m[oy], fe);
            fe = fma(sym_m(a.band, jz, 0), ra0k[oy], fe);
          }
          if (band_hi(jz, K) == P - 1) {
            fm = fma(sym_m(a.band, jz, P - 1), ra8m[oy], fm);
            fe = fma(sym_k(a.band, jz, P - 1), ra8m[oy], fe);
            fe = fma(sym_m(a.band, jz, P - 1), ra8k[oy], fe);
          }
          if (band_lo(jy, K) == 0) {
            fm = fma(sym_m(a.band, jy, 0), c0m, fm);
            fe = fma(sym_k(a.band, jy, 0), c0m, fe);
            fe = fma(sym_m(a.band, jy, 0), c0k, fe);
          }
          if (band_hi(jy, K) == P - 1) {
            fm = fma(sym_m(a.band, jy, P - 1), c8m, fm);
            fe = fma(sym_k(a.band, jy, P - 1), c8m, fe);
            fe = fma(sym_m(a.band, jy, P - 1), c8k, fe);
          }
          FM[oy * CS + lane] = fm;
          FE[oy * CS + lane] = fe;
          BB[oy * CS + lane] = bcur[oy];
        }
      } else {
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
          FM[oy * CS + lane] = fm;
          FE[oy * CS + lane] = fe;
          BB[oy * CS + lane] = bcur[oy];
        }
      }
    }
    __syncthreads();
    // ---- B. lanes = (patch, oy): x contraction, local residual, T^T along x ----
    if (lane < GQ) {
      const int oy = ll;
      T fm[P], fe[P], r[Q];
#pragma unroll
      for (int x = 0; x < P; ++x) {
        fm[x] = FM[oy * CS + c0 + x];
        fe[x] = FE[oy * CS + c0 + x];
      }
      if constexpr (FP) {
        fm[0] += DM[(oz * Q + oy) * F + fl];
        fe[0] += DE[(oz * Q + oy) * F + fl];
        fm[P - 1] += DM[(oz * Q + oy) * F + fl + 1];
        fe[P - 1] += DE[(oz * Q + oy) * F + fl + 1];
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
        r[ox] = BB[oy * CS + c0 + 1 + ox] - s;
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
      for (int mz = 0; mz < Q; ++mz) W[pp * PS + (mx * Q + mz) * Q + oy] = c[mz];
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
      for (int oy = 0; oy < Q; ++oy) v[oy] = W[pp * PS + (mx * Q + mz) * Q + oy];
      fdm_forward<T, K>(a.f, v, c);  // T^T along y
      const T s2 = lmx + a.lam[mz];
#pragma unroll
      for (int my = 0; my < Q; ++my) {
        c[my] *= inv_eig(s2 + a.lam[my]);
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
      for (int y = 0; y < Q; ++y) W[pp * PS + (z * Q + y) * Q + mx] = e[z][y];
  }
  __syncthreads();

  // ---- D. lanes = (patch, y): T along x on the lane's own x lines, in place;
  //      then lanes = (patch, interior column x): store the x rows ----
  if (lane < GQ) {
    const int y = ll;
#pragma unroll
    for (int z = 0; z < Q; ++z) {
      T* w = W + pp * PS + (z * Q + y) * Q;
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
    const unsigned off2 = colb(c0 + 1 + x);
#pragma unroll
    for (int z = 0; z < Q; ++z)
#pragma unroll
      for (int y = 0; y < Q; ++y)
        buf_store<T>(W[pp * PS + (z * Q + y) * Q + x], ur, off2, sbase + splane * (z + 1) + srow * (y + 1));
  }
}

}  // namespace vps
