// Plane-streaming kernels for 3D constant-coefficient level operators: the
// operator A u (and the residual b - A u) and the restriction P^T r.
//
// A workgroup owns an x-y tile of output cells and walks a chunk of cell
// layers along z.  Per input plane it stages the plane's tile (with its x-y
// halo) in LDS, contracts along x and then along y with the banded 1D
// matrices (these are the same for every cell period of a uniform mesh, so a
// work item handles one period of outputs with compile-time coefficients),
// and folds the plane into the z direction in registers with the 1D matrices
// of one z cell: an output plane is final once the last input plane of its
// cell(s) has gone by, and the value on the vertex plane shared by two cells
// is carried from one cell to the next.  Every input plane is read once per
// chunk (plus one halo cell layer at the chunk's start and the x-y halo,
// which neighbouring workgroups read at the same time from L2).
//
// Operator:     A = Kz (x) My (x) Mx + Mz (x) (My (x) Kx + Ky (x) Mx), the
//               Kronecker-sum form of the Laplacian on Cartesian cells
//               (Appendix A.3); per plane the x-y part yields mm = My Mx u and
//               s = My Kx u + Ky Mx u, and the z part is Kz mm + Mz s.
// Restriction:  P^T = Rz (x) Ry (x) Rx with R the transpose of the 1D
//               prolongation (Section 2: the coarse space is embedded in the
//               fine one); fine planes are folded into coarse planes by the
//               1D restriction of one coarse cell.
// Prolongation: u_fine += P e_coarse, P = Pz (x) Py (x) Px; the 2K fine
//               planes of a coarse cell are interpolated from its K+1 coarse
//               planes.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace vps {

// STREAM_RESIDUAL is the operator with the right-hand side subtracted (b - A u); the plain
// operator is a kind of its own so that it holds no right-hand-side registers.
enum StreamKind { STREAM_OPERATOR = 0, STREAM_RESTRICT = 1, STREAM_PROLONG = 2, STREAM_RESIDUAL = 3 };

// Shape of one kind and degree.  In x and y a period of PO outputs reads a
// window of W inputs starting PI inputs after the previous period's.  TX, TY
// periods per tile; ZIN input planes per z cell (the operator and the
// prolongation share the vertex plane between neighbouring cells: K new
// planes per cell; the restriction reads 2K fine planes per coarse cell);
// ZO output planes accumulated per z cell.
template <int KIND, int K>
struct StreamShape {
  static constexpr bool RES = KIND == STREAM_RESIDUAL;
  static constexpr bool OP = KIND == STREAM_OPERATOR || RES;
  static constexpr bool PR = KIND == STREAM_PROLONG;
  static constexpr int PO = PR ? 2 * K : K;
  static constexpr int PI = (KIND == STREAM_RESTRICT) ? 2 * K : K;
  static constexpr int W = OP ? 2 * K + 1 : PR ? K + 1 : 4 * K + 1;
  static constexpr int TX = PR ? ((K == 1) ? 16 : (K == 2) ? 8 : (K == 3) ? 5 : (K == 4) ? 4 : 3)
                               : ((K == 1) ? 32 : (K == 2) ? 16 : (K <= 4) ? 8 : 6);
  static constexpr int TY = PR ? ((K == 1) ? 32 : (K == 2) ? 16 : 8)
                               : ((K == 1) ? 32 : (K == 2) ? 16 : (K == 3) ? 10 : (K == 4) ? 8 : (OP ? 8 : 4));
  static constexpr int NA = OP ? 2 : 1;  // arrays after the x contraction
  static constexpr int ZIN = (KIND == STREAM_RESTRICT) ? 2 * K : K;
  static constexpr int ZO = PR ? 2 * K : K + 1;
  static constexpr int NOX = PO * TX, NOY = PO * TY;
  static constexpr int NIX = PI * (TX - 1) + W, NIY = PI * (TY - 1) + W;
  static constexpr int ITEMS = NOX * TY;  // y-pass work items (x output, y period)
  static constexpr int NIT = (ITEMS + kBlock - 1) / kBlock;
  static constexpr int NPF = (NIX * NIY + kBlock - 1) / kBlock;  // plane elements per thread
  static constexpr int LDS_ELEMS = NIX * NIY + NA * NIY * NOX;
  // nonzero band of period row j inside the window
  static __host__ __device__ constexpr int lo(int j) { return (PR || j == 0) ? 0 : (OP ? K : 2 * K); }
  static __host__ __device__ constexpr int hi(int j) { return OP ? 2 * K : PR ? K : 4 * K; }
};

// The operator's coefficients all come from the two symmetric cell matrices:
// they travel as upper triangles (plus the vertex diagonal summed over its
// two cells), 2 (K+1)(K+2)/2 + 2 scalars instead of 2 K (2K+1) + 2 (K+1)^2,
// so that they stay in scalar registers.  The transfers' come from the 1D
// interpolation of one coarse cell, p[f][c] (fine node f = 0..2K, coarse node
// c = 0..K), whose rows past the middle mirror the first ones
// (p[2K-f][K-c] = p[f][c]): (K+1)^2 scalars.
__host__ __device__ constexpr int cell_sym_idx(int r, int c, int K) {
  return r <= c ? r * (K + 1) - r * (r - 1) / 2 + (c - r) : c * (K + 1) - c * (c - 1) / 2 + (r - c);
}

template <typename T, int KIND, int K>
struct StreamArgs {
  using S = StreamShape<KIND, K>;
  static constexpr int NS = (K + 1) * (K + 2) / 2;
  const T* __restrict__ in;
  const T* __restrict__ b;  // residual only: out = b - A u
  T* __restrict__ out;
  int n1_in, n1_out;
  int ncz;                  // cells of the output grid per direction
  int tiles_x, tiles_y;     // x-y tiles
  int cz;                   // z cells per chunk
  unsigned nblocks;         // tiles_x * tiles_y * chunks
  T pt[S::OP ? 1 : (K + 1) * (K + 1)];       // transfers: p[f][c] for f = 0..K
  T cm[S::OP ? NS : 1], ck[S::OP ? NS : 1];  // operator: upper triangles of the cell mass / stiffness
  T mvv, kvv;                                // operator: the vertex diagonal over both cells

  __device__ T p1(int f, int c) const {
    return f <= K ? pt[f * (K + 1) + c] : pt[(2 * K - f) * (K + 1) + (K - c)];
  }

  // period row j, window entry i of the x-y contraction: mass (t = 0) / stiffness (t = 1)
  // for the operator (the vertex row j = 0 spans both cells, j > 0 the cell after it),
  // the transfer rows otherwise
  __device__ T g(int t, int j, int i) const {
    if constexpr (S::OP) {
      const T* c = t == 0 ? cm : ck;
      if (j > 0) return c[cell_sym_idx(j, i - K, K)];
      if (i < K) return c[cell_sym_idx(K, i, K)];
      if (i > K) return c[cell_sym_idx(0, i - K, K)];
      return t == 0 ? mvv : kvv;
    } else if constexpr (S::PR) {
      return p1(j, i);  // fine row j of the period, coarse node i
    } else {
      // coarse row j of the period (j = 0: the vertex between two coarse cells), fine node i of the window
      if (j > 0) return p1(i - 2 * K, j);
      return i <= 2 * K ? p1(i, K) : p1(i - 2 * K, 0);
    }
  }
  // z fold: entry [out o][in l] of the cell matrix (operator) or cell block (transfers)
  __device__ T z(int t, int o, int l) const {
    if constexpr (S::OP) return (t == 0 ? cm : ck)[cell_sym_idx(o, l, K)];
    else if constexpr (S::PR) return p1(o, l);  // fine plane o of the coarse cell from coarse plane l
    else return p1(l, o);                       // coarse plane o from fine plane l of the coarse cell
  }
};

template <typename T>
__device__ inline T ld_or_zero(const T* __restrict__ p, size_t i, bool ok) {
  return ok ? p[i] : T(0);
}

template <typename T, int KIND, int K>
__global__ void __launch_bounds__(kBlock) stream3_kernel(const StreamArgs<T, KIND, K> a) {
  using S = StreamShape<KIND, K>;
  constexpr bool OP = S::OP;
  constexpr int PO = S::PO, PI = S::PI, W = S::W, TX = S::TX, TY = S::TY, NA = S::NA, ZIN = S::ZIN;
  constexpr int NOX = S::NOX, NIX = S::NIX, NIY = S::NIY, NIT = S::NIT, NPF = S::NPF;
  __shared__ T U[NIY * NIX];
  __shared__ T XA[NA * NIY * NOX];

  // XCD-aware order: each of the 8 XCDs runs one contiguous range of blocks
  const unsigned h = blockIdx.x;
  const unsigned per = gridDim.x / kXcd;
  const unsigned logical = (h % kXcd) * per + h / kXcd;
  if (logical >= a.nblocks) return;
  const int t = threadIdx.x;
  const int tx = (int)(logical % (unsigned)a.tiles_x);
  const unsigned rest = logical / (unsigned)a.tiles_x;
  const int ty = (int)(rest % (unsigned)a.tiles_y);
  const int chunk = (int)(rest / (unsigned)a.tiles_y);
  const int cz0 = chunk * a.cz;
  const int cz1 = min(a.ncz, cz0 + a.cz);
  // first cell walked: one halo cell before the chunk (the prolongation needs none)
  const int cs = S::PR ? cz0 : max(cz0 - 1, 0);

  const int n1i = a.n1_in, n1o = a.n1_out;
  const size_t pin = (size_t)n1i * n1i, pout = (size_t)n1o * n1o;
  constexpr int HALO = S::PR ? 0 : PI;  // input nodes left of the tile's first output period
  const int in0x = PI * TX * tx - HALO, in0y = PI * TY * ty - HALO;
  const int out0x = PO * TX * tx, out0y = PO * TY * ty;

  // this thread's elements of the input tile (plane offsets, in-grid flags)
  unsigned pf_off[NPF];
  bool pf_ok[NPF];
#pragma unroll
  for (int m = 0; m < NPF; ++m) {
    const int e = t + kBlock * m;
    const int x = e % NIX, y = e / NIX;
    const int gx = in0x + x, gy = in0y + y;
    pf_ok[m] = e < NIX * NIY && gx >= 0 && gx < n1i && gy >= 0 && gy < n1i;
    pf_off[m] = pf_ok[m] ? (unsigned)(gy * n1i + gx) : 0u;
  }
  // this thread's output columns: items (xo, py), rows yo = py * PO + j
  int it_xo[NIT], it_py[NIT];
  bool it_ok[NIT];
#pragma unroll
  for (int m = 0; m < NIT; ++m) {
    const int it = t + kBlock * m;
    it_ok[m] = it < S::ITEMS;
    it_xo[m] = it % NOX;
    it_py[m] = it / NOX;
  }

  // prefetch registers: the next input plane's tile elements (and b of the next plane for the residual)
  T pf[NPF];
  constexpr int NB = S::RES ? NIT : 1, PB = S::RES ? PO : 1;
  T pb[NB][PB];
  auto prefetch = [&](int p) {
    const T* src = a.in + (size_t)p * pin;
#pragma unroll
    for (int m = 0; m < NPF; ++m) pf[m] = ld_or_zero(src, pf_off[m], pf_ok[m]);
    if constexpr (S::RES) {
      {
        const T* bs = a.b + (size_t)p * pout;
#pragma unroll
        for (int m = 0; m < NIT; ++m)
#pragma unroll
          for (int j = 0; j < PO; ++j) {
            const int gx = out0x + it_xo[m], gy = out0y + it_py[m] * PO + j;
            const bool ok = it_ok[m] && gx < n1o && gy < n1o;
            pb[m][j] = ld_or_zero(bs, ok ? (size_t)gy * n1o + gx : 0, ok);
          }
      }
    }
  };

  // x-y contraction of the plane held in pf; the next plane's loads are issued first.
  // Results: v0 (operator: mm = My Mx u; restriction: Ry Rx r), v1 (operator: s).
  T v0[NIT][PO], v1[NIT][PO], cb[NB][PB];
  auto plane = [&](int p, int plast) {
#pragma unroll
    for (int m = 0; m < NPF; ++m)
      if (t + kBlock * m < NIX * NIY) U[t + kBlock * m] = pf[m];
    if constexpr (S::RES) {
#pragma unroll
      for (int m = 0; m < NIT; ++m)
#pragma unroll
        for (int j = 0; j < PO; ++j) cb[m][j] = pb[m][j];
    }
    if (p < plast) prefetch(p + 1);
    __syncthreads();
    // x: items (px, yi), outputs px * PO + j of row yi
    for (int w = t; w < TX * NIY; w += kBlock) {
      const int px = w % TX, yi = w / TX;
      T u[W];
#pragma unroll
      for (int i = 0; i < W; ++i) u[i] = U[yi * NIX + px * PI + i];
#pragma unroll
      for (int j = 0; j < PO; ++j) {
        T s0 = T(0), s1 = T(0);
#pragma unroll
        for (int i = S::lo(j); i <= S::hi(j); ++i) {
          s0 = fma(a.g(0, j, i), u[i], s0);
          if constexpr (OP) s1 = fma(a.g(1, j, i), u[i], s1);
        }
        XA[yi * NOX + px * PO + j] = s0;
        if constexpr (OP) XA[NIY * NOX + yi * NOX + px * PO + j] = s1;
      }
    }
    __syncthreads();
    // y: items (xo, py), outputs rows py * PO + j
#pragma unroll
    for (int m = 0; m < NIT; ++m) {
      if (!it_ok[m]) continue;
      const int xo = it_xo[m], row0 = it_py[m] * PI;
      T x0[W], x1[W];
#pragma unroll
      for (int i = 0; i < W; ++i) {
        x0[i] = XA[(row0 + i) * NOX + xo];
        if constexpr (OP) x1[i] = XA[NIY * NOX + (row0 + i) * NOX + xo];
      }
#pragma unroll
      for (int j = 0; j < PO; ++j) {
        T s0 = T(0), s1 = T(0);
#pragma unroll
        for (int i = S::lo(j); i <= S::hi(j); ++i) {
          s0 = fma(a.g(0, j, i), x0[i], s0);
          if constexpr (OP) {
            s1 = fma(a.g(0, j, i), x1[i], s1);
            s1 = fma(a.g(1, j, i), x0[i], s1);
          }
        }
        v0[m][j] = s0;
        if constexpr (OP) v1[m][j] = s1;
      }
    }
  };

  // write one output plane from acc[.][.][q]
  T acc[NIT][PO][S::ZO];
  auto emit = [&](int zp, int q) {
    const bool zdir = zp == 0 || zp == n1o - 1;
    T* dst = a.out + (size_t)zp * pout;
#pragma unroll
    for (int m = 0; m < NIT; ++m) {
      if (!it_ok[m]) continue;
      const int gx = out0x + it_xo[m];
#pragma unroll
      for (int j = 0; j < PO; ++j) {
        const int gy = out0y + it_py[m] * PO + j;
        if (gx >= n1o || gy >= n1o) continue;
        const bool dir = zdir || gx == 0 || gx == n1o - 1 || gy == 0 || gy == n1o - 1;
        dst[(size_t)gy * n1o + gx] = dir ? T(0) : acc[m][j][q];
        // the last grid line of each direction lies outside every tile: written by its neighbour
        if (gx == n1o - 2) dst[(size_t)gy * n1o + gx + 1] = T(0);
        if (gy == n1o - 2) dst[(size_t)(gy + 1) * n1o + gx] = T(0);
        if (gx == n1o - 2 && gy == n1o - 2) dst[(size_t)(gy + 1) * n1o + gx + 1] = T(0);
      }
    }
  };
  auto emit_zero_plane = [&](int zp) {
    T* dst = a.out + (size_t)zp * pout;
#pragma unroll
    for (int m = 0; m < NIT; ++m) {
      if (!it_ok[m]) continue;
      const int gx = out0x + it_xo[m];
#pragma unroll
      for (int j = 0; j < PO; ++j) {
        const int gy = out0y + it_py[m] * PO + j;
        if (gx >= n1o || gy >= n1o) continue;
        dst[(size_t)gy * n1o + gx] = T(0);
        if (gx == n1o - 2) dst[(size_t)gy * n1o + gx + 1] = T(0);
        if (gy == n1o - 2) dst[(size_t)(gy + 1) * n1o + gx] = T(0);
        if (gx == n1o - 2 && gy == n1o - 2) dst[(size_t)(gy + 1) * n1o + gx + 1] = T(0);
      }
    }
  };

  constexpr bool resid = S::RES;
  if constexpr (OP) {
    // planes K*cs .. K*cz1; the vertex plane of each cell is folded into both of its cells
    const int plast = K * cz1;
    prefetch(K * cs);
    plane(K * cs, plast);
    T pm[NIT][PO], ps[NIT][PO];
#pragma unroll
    for (int m = 0; m < NIT; ++m)
#pragma unroll
      for (int j = 0; j < PO; ++j) {
        pm[m][j] = v0[m][j];
        ps[m][j] = v1[m][j];
#pragma unroll
        for (int i = 0; i <= K; ++i) acc[m][j][i] = T(0);
      }
    for (int c = cs; c < cz1; ++c) {
      // start cell c: carry (acc[.][.][K] of cell c-1) plus its first plane
#pragma unroll
      for (int m = 0; m < NIT; ++m)
#pragma unroll
        for (int j = 0; j < PO; ++j) {
          const T carry = acc[m][j][K];
#pragma unroll
          for (int i = 0; i <= K; ++i)
            acc[m][j][i] = fma(a.z(1, i, 0), pm[m][j], a.z(0, i, 0) * ps[m][j]);
          acc[m][j][0] += carry;
          if constexpr (resid) acc[m][j][0] -= cb[m][j];
        }
#pragma unroll
      for (int l = 1; l <= K; ++l) {
        plane(K * c + l, plast);
#pragma unroll
        for (int m = 0; m < NIT; ++m)
#pragma unroll
          for (int j = 0; j < PO; ++j) {
#pragma unroll
            for (int i = 0; i <= K; ++i)
              acc[m][j][i] = fma(a.z(1, i, l), v0[m][j], fma(a.z(0, i, l), v1[m][j], acc[m][j][i]));
            if constexpr (resid) {
              if (l < K) acc[m][j][l] -= cb[m][j];
            }
          }
      }
      // the vertex plane K*(c+1) also starts cell c+1
#pragma unroll
      for (int m = 0; m < NIT; ++m)
#pragma unroll
        for (int j = 0; j < PO; ++j) {
          pm[m][j] = v0[m][j];
          ps[m][j] = v1[m][j];
        }
      if (c >= cz0) {
        if constexpr (resid) {
#pragma unroll
          for (int m = 0; m < NIT; ++m)
#pragma unroll
            for (int j = 0; j < PO; ++j)
#pragma unroll
              for (int i = 0; i < K; ++i) acc[m][j][i] = -acc[m][j][i];
        }
#pragma unroll
        for (int i = 0; i < K; ++i) emit(K * c + i, i);
      }
      // the b of plane K*(c+1) is subtracted when cell c+1 starts
    }
    if (cz1 == a.ncz) emit_zero_plane(K * a.ncz);
  } else if constexpr (S::PR) {
    // coarse planes K*cz0 .. K*cz1; fine planes 2K*c + j (j < 2K) from the K+1 planes of coarse cell c
    const int plast = K * cz1;
    prefetch(K * cs);
    plane(K * cs, plast);
    T pv[NIT][PO];
#pragma unroll
    for (int m = 0; m < NIT; ++m)
#pragma unroll
      for (int j = 0; j < PO; ++j) pv[m][j] = v0[m][j];
    for (int c = cs; c < cz1; ++c) {
#pragma unroll
      for (int m = 0; m < NIT; ++m)
#pragma unroll
        for (int j = 0; j < PO; ++j)
#pragma unroll
          for (int q = 0; q < 2 * K; ++q) acc[m][j][q] = a.z(0, q, 0) * pv[m][j];
#pragma unroll
      for (int l = 1; l <= K; ++l) {
        plane(K * c + l, plast);
#pragma unroll
        for (int m = 0; m < NIT; ++m)
#pragma unroll
          for (int j = 0; j < PO; ++j)
#pragma unroll
            for (int q = 0; q < 2 * K; ++q) acc[m][j][q] = fma(a.z(0, q, l), v0[m][j], acc[m][j][q]);
      }
#pragma unroll
      for (int m = 0; m < NIT; ++m)
#pragma unroll
        for (int j = 0; j < PO; ++j) pv[m][j] = v0[m][j];
      // add to the fine planes; Dirichlet nodes keep their (zero) value
#pragma unroll
      for (int q = 0; q < 2 * K; ++q) {
        const int zf = 2 * K * c + q;
        if (zf == 0) continue;
        T* dst = a.out + (size_t)zf * pout;
#pragma unroll
        for (int m = 0; m < NIT; ++m) {
          if (!it_ok[m]) continue;
          const int gx = out0x + it_xo[m];
          if (gx == 0 || gx >= n1o - 1) continue;
#pragma unroll
          for (int j = 0; j < PO; ++j) {
            const int gy = out0y + it_py[m] * PO + j;
            if (gy == 0 || gy >= n1o - 1) continue;
            dst[(size_t)gy * n1o + gx] += acc[m][j][q];
          }
        }
      }
    }
  } else {
    // fine planes 2K*cs .. 2K*cz1 - 1, each inside one coarse cell
    const int plast = 2 * K * cz1 - 1;
    prefetch(2 * K * cs);
#pragma unroll
    for (int m = 0; m < NIT; ++m)
#pragma unroll
      for (int j = 0; j < PO; ++j)
#pragma unroll
        for (int i = 0; i <= K; ++i) acc[m][j][i] = T(0);
    for (int c = cs; c < cz1; ++c) {
#pragma unroll
      for (int l = 0; l < 2 * K; ++l) {
        plane(2 * K * c + l, plast);
#pragma unroll
        for (int m = 0; m < NIT; ++m)
#pragma unroll
          for (int j = 0; j < PO; ++j) {
            if (l == 0) {
              const T carry = acc[m][j][K];
#pragma unroll
              for (int i = 0; i <= K; ++i) acc[m][j][i] = a.z(0, i, 0) * v0[m][j];
              acc[m][j][0] += carry;
            } else {
#pragma unroll
              for (int i = 0; i <= K; ++i) acc[m][j][i] = fma(a.z(0, i, l), v0[m][j], acc[m][j][i]);
            }
          }
      }
      if (c >= cz0) {
#pragma unroll
        for (int i = 0; i < K; ++i) emit(K * c + i, i);
      }
    }
    if (cz1 == a.ncz) emit_zero_plane(K * a.ncz);
  }
}

}  // namespace vps
