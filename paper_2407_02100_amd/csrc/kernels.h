// Device kernels of libvps (HIP, gfx950).  Library-internal header.
//
// Storage: a level vector is the full nodal grid of (k N + 1)^d values,
// x fastest; Dirichlet entries are 0.  Every kernel below works on boxes of
// that grid staged in LDS and applies 1D operators along one direction at a
// time (sum factorisation, Appendix A.1): the Laplacian on a Cartesian cell
// is the Kronecker sum of 1D mass and stiffness matrices (Appendix A.3), and
// the transfer operators are Kronecker products of the 1D prolongation.
#pragma once

#include <hip/hip_runtime.h>

namespace vps {

constexpr int kBlock = 256;
// XCDs of the MI355X: workgroup ids are dealt round-robin over them, and each has its own L2.
constexpr int kXcd = 8;

// ---------------------------------------------------------------------------
// 1D band structure.  Nodes are numbered so that cell boundaries sit at
// multiples of K.  A node interior to a cell couples to the K+1 nodes of that
// cell; a cell vertex couples to the 2K+1 nodes of its two cells.
__host__ __device__ constexpr int band_lo(int j, int K) { return (j % K == 0) ? j - K : j - j % K; }
__host__ __device__ constexpr int band_hi(int j, int K) { return (j % K == 0) ? j + K : j - j % K + K; }

// Same band restricted to the cell [h K, h K + K] (h = 0 or 1): the part of
// row j contributed by that cell, empty (lo > hi) if j is not in it.
__host__ __device__ constexpr int half_lo(int j, int K, int h) {
  return (j >= h * K && j <= h * K + K) ? h * K : 1;
}
__host__ __device__ constexpr int half_hi(int j, int K, int h) {
  return (j >= h * K && j <= h * K + K) ? h * K + K : 0;
}

// ---------------------------------------------------------------------------
// Patch smoother (Algorithm 4 per color).

template <typename T, int K>
struct PatchMats {
  static constexpr int P = 2 * K + 1;  // closure nodes per direction
  static constexpr int Q = 2 * K - 1;  // interior nodes per direction
  // Interior rows of the 2-cell 1D patch mass/stiffness matrices (Q x P,
  // row-major, row o <-> closure node o+1).  Constant coefficient: [0] holds
  // the full matrix.  Cell coefficient: [h] holds the part of cell h.
  T M[2][Q * P];
  T Kst[2][Q * P];
  // Fast diagonalisation: T_1D (Q x Q, T[i*Q+m] = component i of mode m),
  // eigenvalues of the interior 1D patch problem.
  T T1[Q * Q];
  T lam[Q];
};

template <typename T, int K>
struct PatchArgs {
  T* __restrict__ u;
  const T* __restrict__ b;
  const T* __restrict__ rho;       // per cell of the level (cell coefficient modes)
  const float* __restrict__ scal;  // per patch x Q^d eigenmode factors (learned mode)
  int n1;                          // nodes per direction
  int ncell;                       // cells per direction
  int v0[3];                       // first vertex of this color, per direction
  int np[3];                       // patches of this color, per direction
  PatchMats<T, K> m;
};

// coef: 0 constant, 1 cell coefficient + patch-mean FDM, 2 as 1 with learned scaling
template <typename T, int K, int D, int COEF, int PB>
struct PatchKernelShape {
  static constexpr int P = 2 * K + 1, Q = 2 * K - 1;
  static constexpr int NX = 2 * K * PB + 1;  // closure box extent along x
  static constexpr int QX = PB * Q;          // interiors concatenated along x
  static constexpr int NH = (COEF == 0) ? 1 : 2;
  static constexpr int PD2 = (D == 3) ? P : 1;
  static constexpr int QD2 = (D == 3) ? Q : 1;
  static constexpr int BOX = PD2 * P * NX;
  static constexpr int XS = 2 * NH * PD2 * P * QX;               // after the x contraction
  static constexpr int YS = (D == 3) ? 2 * NH * NH * P * Q * QX : 0;  // after the y contraction (3D)
  static constexpr int RS = QD2 * Q * QX;                         // one interior array
  // 3D keeps the interior arrays in buf1 (X is dead once G exists), 2D in
  // buf0 (the box is dead once X exists).
  static constexpr int BUF0 = (D == 3) ? (BOX > YS ? BOX : YS) : (BOX > 2 * RS ? BOX : 2 * RS);
  static constexpr int BUF1 = (D == 3) ? (XS > 2 * RS ? XS : 2 * RS) : XS;
  static constexpr int LDS_BYTES = (BUF0 + BUF1) * (int)sizeof(T);
};

template <typename T, int K, int D, int COEF, int PB>
__global__ void __launch_bounds__(kBlock) patch_color_kernel(const PatchArgs<T, K> a) {
  using Sh = PatchKernelShape<T, K, D, COEF, PB>;
  constexpr int P = Sh::P, Q = Sh::Q, NX = Sh::NX, QX = Sh::QX, NH = Sh::NH;
  __shared__ T buf0[Sh::BUF0];
  __shared__ T buf1[Sh::BUF1];
  __shared__ T rho_s[PB][1 << D];
  __shared__ T rbar_s[PB];

  const int tid = threadIdx.x;
  const int bx = blockIdx.x;
  const int py = (D == 3) ? blockIdx.y : blockIdx.y;
  const int pz = (D == 3) ? blockIdx.z : 0;
  const int first = bx * PB;
  const int nvalid = min(PB, a.np[0] - first);
  const int vx0 = a.v0[0] + 2 * first;
  const int vy = a.v0[1] + 2 * py;
  const int vz = (D == 3) ? a.v0[2] + 2 * pz : 1;
  const int n1 = a.n1;
  const int x0 = K * (vx0 - 1);
  const int y0 = K * (vy - 1);
  const int z0 = (D == 3) ? K * (vz - 1) : 0;
  const int xend = K * (vx0 - 1 + 2 * nvalid);  // last closure node of the last valid patch

  // --- coefficient of the patches' cells ---
  if (COEF != 0) {
    for (int w = tid; w < PB * (1 << D); w += kBlock) {
      const int m = w >> D, c = w & ((1 << D) - 1);
      T v = T(1);
      if (m < nvalid) {
        const int cx = vx0 + 2 * m - 1 + (c & 1);
        const int cy = vy - 1 + ((c >> 1) & 1);
        const int cz = (D == 3) ? vz - 1 + ((c >> 2) & 1) : 0;
        v = a.rho[cx + a.ncell * (cy + a.ncell * cz)];
      }
      rho_s[m][c] = v;
    }
    __syncthreads();
    if (tid < PB) {
      T s = T(0);
      for (int c = 0; c < (1 << D); ++c) s += rho_s[tid][c];
      rbar_s[tid] = s / T(1 << D);
    }
  }

  // --- gather the closure box ---
  T* box = buf0;
  for (int w = tid; w < Sh::BOX; w += kBlock) {
    const int x = w % NX;
    const int yz = w / NX;
    const int y = yz % P;
    const int z = yz / P;
    const int gx = x0 + x;
    T v = T(0);
    if (gx <= xend) v = a.u[(size_t)gx + (size_t)n1 * ((size_t)(y0 + y) + (size_t)n1 * (size_t)(z0 + z))];
    box[w] = v;
  }
  __syncthreads();

  // --- x contraction: Xm[h] = M_x^h ubar, Xk[h] = K_x^h ubar (lines (z,y,m)) ---
  // layout: X[(h*2 + {0:M,1:K})][z][y][i]
  T* X = buf1;
  constexpr int XA = Sh::PD2 * P * QX;
  for (int w = tid; w < Sh::PD2 * P * PB; w += kBlock) {
    const int m = w % PB;
    const int yz = w / PB;
    if (m >= nvalid) continue;
    T v[P];
#pragma unroll
    for (int i = 0; i < P; ++i) v[i] = box[yz * NX + 2 * K * m + i];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
#pragma unroll
      for (int o = 0; o < Q; ++o) {
        const int j = o + 1;
        const int lo = (COEF == 0) ? band_lo(j, K) : half_lo(j, K, h);
        const int hi = (COEF == 0) ? band_hi(j, K) : half_hi(j, K, h);
        T am = T(0), ak = T(0);
#pragma unroll
        for (int i = 0; i < P; ++i) {
          if (i < lo || i > hi) continue;
          am += a.m.M[h][o * P + i] * v[i];
          ak += a.m.Kst[h][o * P + i] * v[i];
        }
        X[(h * 2 + 0) * XA + yz * QX + m * Q + o] = am;
        X[(h * 2 + 1) * XA + yz * QX + m * Q + o] = ak;
      }
    }
  }
  __syncthreads();

  T* R0 = (D == 3) ? buf1 : buf0;
  T* R1 = R0 + Sh::RS;

  if constexpr (D == 3) {
    // --- y contraction (lines (z, i)) ---
    // G[(hx*NH + hy)*2 + {0,1}][z][y'][i]:
    //   G0 = M_y^hy Xk^hx + K_y^hy Xm^hx   (terms with K along x or y)
    //   G1 = M_y^hy Xm^hx                  (the term that takes K along z)
    T* G = buf0;
    constexpr int GA = P * Q * QX;
    for (int w = tid; w < P * QX; w += kBlock) {
      const int i = w % QX;
      const int z = w / QX;
      if (i / Q >= nvalid) continue;
#pragma unroll
      for (int hx = 0; hx < NH; ++hx) {
        T xm[P], xk[P];
#pragma unroll
        for (int y = 0; y < P; ++y) {
          xm[y] = X[(hx * 2 + 0) * XA + (z * P + y) * QX + i];
          xk[y] = X[(hx * 2 + 1) * XA + (z * P + y) * QX + i];
        }
#pragma unroll
        for (int hy = 0; hy < NH; ++hy) {
#pragma unroll
          for (int o = 0; o < Q; ++o) {
            const int j = o + 1;
            const int lo = (COEF == 0) ? band_lo(j, K) : half_lo(j, K, hy);
            const int hi = (COEF == 0) ? band_hi(j, K) : half_hi(j, K, hy);
            T g0 = T(0), g1 = T(0);
#pragma unroll
            for (int y = 0; y < P; ++y) {
              if (y < lo || y > hi) continue;
              g0 += a.m.M[hy][o * P + y] * xk[y] + a.m.Kst[hy][o * P + y] * xm[y];
              g1 += a.m.M[hy][o * P + y] * xm[y];
            }
            G[((hx * NH + hy) * 2 + 0) * GA + (z * Q + o) * QX + i] = g0;
            G[((hx * NH + hy) * 2 + 1) * GA + (z * Q + o) * QX + i] = g1;
          }
        }
      }
    }
    __syncthreads();

    // --- z contraction and local residual (lines (y', i)): R0 = b - Abar ubar ---
    for (int w = tid; w < Q * QX; w += kBlock) {
      const int i = w % QX;
      const int yo = w / QX;
      const int m = i / Q;
      if (m >= nvalid) continue;
      T acc[Q];
#pragma unroll
      for (int o = 0; o < Q; ++o) acc[o] = T(0);
#pragma unroll
      for (int hz = 0; hz < NH; ++hz) {
        // fold the cell coefficient of the cells (hx, hy, hz) into the y results
        T g0[P], g1[P];
#pragma unroll
        for (int z = 0; z < P; ++z) {
          T s0 = T(0), s1 = T(0);
#pragma unroll
          for (int hx = 0; hx < NH; ++hx)
#pragma unroll
            for (int hy = 0; hy < NH; ++hy) {
              const T r = (COEF == 0) ? T(1) : rho_s[m][hx + 2 * hy + 4 * hz];
              s0 += r * G[((hx * NH + hy) * 2 + 0) * GA + (z * Q + yo) * QX + i];
              s1 += r * G[((hx * NH + hy) * 2 + 1) * GA + (z * Q + yo) * QX + i];
            }
          g0[z] = s0;
          g1[z] = s1;
        }
#pragma unroll
        for (int o = 0; o < Q; ++o) {
          const int j = o + 1;
          const int lo = (COEF == 0) ? band_lo(j, K) : half_lo(j, K, hz);
          const int hi = (COEF == 0) ? band_hi(j, K) : half_hi(j, K, hz);
#pragma unroll
          for (int z = 0; z < P; ++z) {
            if (z < lo || z > hi) continue;
            acc[o] += a.m.M[hz][o * P + z] * g0[z] + a.m.Kst[hz][o * P + z] * g1[z];
          }
        }
      }
      const int gx = K * (vx0 + 2 * m - 1) + 1 + (i - m * Q);
      const int gy = y0 + 1 + yo;
#pragma unroll
      for (int o = 0; o < Q; ++o) {
        const int gz = z0 + 1 + o;
        const T bv = a.b[(size_t)gx + (size_t)n1 * ((size_t)gy + (size_t)n1 * (size_t)gz)];
        R0[(o * Q + yo) * QX + i] = bv - acc[o];
      }
    }
    __syncthreads();
  } else {
    // --- 2D: y contraction and local residual (lines i) ---
    for (int w = tid; w < QX; w += kBlock) {
      const int i = w;
      const int m = i / Q;
      if (m >= nvalid) continue;
      T acc[Q];
#pragma unroll
      for (int o = 0; o < Q; ++o) acc[o] = T(0);
#pragma unroll
      for (int hy = 0; hy < NH; ++hy) {
        T xm[P], xk[P];
#pragma unroll
        for (int y = 0; y < P; ++y) {
          T s0 = T(0), s1 = T(0);
#pragma unroll
          for (int hx = 0; hx < NH; ++hx) {
            const T r = (COEF == 0) ? T(1) : rho_s[m][hx + 2 * hy];
            s0 += r * X[(hx * 2 + 0) * XA + y * QX + i];
            s1 += r * X[(hx * 2 + 1) * XA + y * QX + i];
          }
          xm[y] = s0;
          xk[y] = s1;
        }
#pragma unroll
        for (int o = 0; o < Q; ++o) {
          const int j = o + 1;
          const int lo = (COEF == 0) ? band_lo(j, K) : half_lo(j, K, hy);
          const int hi = (COEF == 0) ? band_hi(j, K) : half_hi(j, K, hy);
#pragma unroll
          for (int y = 0; y < P; ++y) {
            if (y < lo || y > hi) continue;
            acc[o] += a.m.M[hy][o * P + y] * xk[y] + a.m.Kst[hy][o * P + y] * xm[y];
          }
        }
      }
      const int gx = K * (vx0 + 2 * m - 1) + 1 + (i - m * Q);
#pragma unroll
      for (int o = 0; o < Q; ++o) {
        const int gy = y0 + 1 + o;
        R0[o * QX + i] = a.b[(size_t)gx + (size_t)n1 * (size_t)gy] - acc[o];
      }
    }
    __syncthreads();
  }

  // --- fast diagonalisation (eq:fdm:inverse): d = S diag(s) S^T r ---
  // Stage A: R1 = T^T along x.
  constexpr int NL = Sh::QD2 * Q;  // lines per patch per direction
  for (int w = tid; w < NL * PB; w += kBlock) {
    const int m = w % PB;
    const int l = w / PB;
    if (m >= nvalid) continue;
    T v[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = R0[l * QX + m * Q + i];
#pragma unroll
    for (int mo = 0; mo < Q; ++mo) {
      T s = T(0);
#pragma unroll
      for (int i = 0; i < Q; ++i) s += a.m.T1[i * Q + mo] * v[i];
      R1[l * QX + m * Q + mo] = s;
    }
  }
  __syncthreads();
  // Stage B: T^T along y (R1 -> R0); in 2D also scale.
  for (int w = tid; w < Sh::QD2 * QX; w += kBlock) {
    const int i = w % QX;
    const int z = w / QX;
    const int m = i / Q;
    if (m >= nvalid) continue;
    T v[Q];
#pragma unroll
    for (int y = 0; y < Q; ++y) v[y] = R1[(z * Q + y) * QX + i];
#pragma unroll
    for (int mo = 0; mo < Q; ++mo) {
      T s = T(0);
#pragma unroll
      for (int y = 0; y < Q; ++y) s += a.m.T1[y * Q + mo] * v[y];
      if (D == 2) {
        const int mx = i - m * Q;
        T lam = a.m.lam[mx] + a.m.lam[mo];
        T f = T(1);
        if (COEF != 0) lam *= rbar_s[m];
        if (COEF == 2) {
          const long long pid = (long long)(vx0 + 2 * m - 1) + (long long)(a.ncell - 1) * (vy - 1);
          f = (T)a.scal[pid * (Q * Q) + mx + Q * mo];
        }
        s = s * f / lam;
      }
      R0[(z * Q + mo) * QX + i] = s;
    }
  }
  __syncthreads();
  if constexpr (D == 3) {
    // Stage C: T^T along z, scale, T along z (lines (y, i)), R0 -> R1.
    for (int w = tid; w < Q * QX; w += kBlock) {
      const int i = w % QX;
      const int y = w / QX;
      const int m = i / Q;
      if (m >= nvalid) continue;
      const int mx = i - m * Q;
      T v[Q], c[Q];
#pragma unroll
      for (int z = 0; z < Q; ++z) v[z] = R0[(z * Q + y) * QX + i];
      long long pid = 0;
      if (COEF == 2)
        pid = (long long)(vx0 + 2 * m - 1) +
              (long long)(a.ncell - 1) * ((long long)(vy - 1) + (long long)(a.ncell - 1) * (vz - 1));
#pragma unroll
      for (int mz = 0; mz < Q; ++mz) {
        T s = T(0);
#pragma unroll
        for (int z = 0; z < Q; ++z) s += a.m.T1[z * Q + mz] * v[z];
        T lam = a.m.lam[mx] + a.m.lam[y] + a.m.lam[mz];
        T f = T(1);
        if (COEF != 0) lam *= rbar_s[m];
        if (COEF == 2) f = (T)a.scal[pid * (Q * Q * Q) + mx + Q * (y + Q * mz)];
        c[mz] = s * f / lam;
      }
#pragma unroll
      for (int z = 0; z < Q; ++z) {
        T s = T(0);
#pragma unroll
        for (int mz = 0; mz < Q; ++mz) s += a.m.T1[z * Q + mz] * c[mz];
        R1[(z * Q + y) * QX + i] = s;
      }
    }
    __syncthreads();
  }
  T* RY = (D == 3) ? R1 : R0;  // current input of the y back-transform
  T* RX = (D == 3) ? R0 : R1;
  // Stage D: T along y.
  for (int w = tid; w < Sh::QD2 * QX; w += kBlock) {
    const int i = w % QX;
    const int z = w / QX;
    if (i / Q >= nvalid) continue;
    T v[Q];
#pragma unroll
    for (int my = 0; my < Q; ++my) v[my] = RY[(z * Q + my) * QX + i];
#pragma unroll
    for (int y = 0; y < Q; ++y) {
      T s = T(0);
#pragma unroll
      for (int my = 0; my < Q; ++my) s += a.m.T1[y * Q + my] * v[my];
      RX[(z * Q + y) * QX + i] = s;
    }
  }
  __syncthreads();
  // Stage E: T along x, add to the gathered interior, scatter (eq:scatter).
  for (int w = tid; w < NL * PB; w += kBlock) {
    const int m = w % PB;
    const int l = w / PB;
    if (m >= nvalid) continue;
    T v[Q];
#pragma unroll
    for (int mx = 0; mx < Q; ++mx) v[mx] = RX[l * QX + m * Q + mx];
    const int yo = l % Q;
    const int zo = l / Q;
    const size_t rowbase = (size_t)(K * (vx0 + 2 * m - 1) + 1) +
                           (size_t)n1 * ((size_t)(y0 + 1 + yo) + (size_t)n1 * (size_t)(D == 3 ? z0 + 1 + zo : 0));
#pragma unroll
    for (int x = 0; x < Q; ++x) {
      T s = T(0);
#pragma unroll
      for (int mx = 0; mx < Q; ++mx) s += a.m.T1[x * Q + mx] * v[mx];
      a.u[rowbase + x] += s;
    }
  }
}

// ---------------------------------------------------------------------------
// Tile kernels: operator (constant coefficient) and transfers.
//
// A tile covers TC cells per direction.  Out[o] = sum_i G[o][i] In[i] along
// each direction, with G a NO x NI block of a banded 1D matrix that is the
// same for every tile (translation invariance of the uniform mesh).

enum TileKind { TILE_OPERATOR = 0, TILE_RESTRICT = 1, TILE_PROLONG = 2 };

template <int KIND, int K, int TC>
struct TileShape;
template <int K, int TC>
struct TileShape<TILE_OPERATOR, K, TC> {
  static constexpr int NO = K * TC, NI = K * (TC + 1) + 1, OUT_SCALE = 1, IN_OFF = -K;
  // output o <-> input node o + K (cell boundaries at multiples of K)
  static __host__ __device__ constexpr int lo(int o) { return band_lo(o + K, K); }
  static __host__ __device__ constexpr int hi(int o) { return band_hi(o + K, K); }
};
template <int K, int TC>
struct TileShape<TILE_RESTRICT, K, TC> {
  // coarse outputs [K c0, K (c0+TC)), fine inputs [2K (c0-1), 2K (c0+TC)]
  static constexpr int NO = K * TC, NI = 2 * K * (TC + 1) + 1;
  static __host__ __device__ constexpr int lo(int o) {
    return ((o + K) % K == 0) ? 2 * K * ((o + K) / K - 1) : 2 * K * ((o + K) / K);
  }
  static __host__ __device__ constexpr int hi(int o) {
    return ((o + K) % K == 0) ? 2 * K * ((o + K) / K + 1) : 2 * K * ((o + K) / K) + 2 * K;
  }
};
template <int K, int TC>
struct TileShape<TILE_PROLONG, K, TC> {
  // fine outputs [2K c0, 2K (c0+TC)), coarse inputs [K c0, K (c0+TC)]
  static constexpr int NO = 2 * K * TC, NI = K * TC + 1;
  static __host__ __device__ constexpr int lo(int o) { return K * (o / (2 * K)); }
  static __host__ __device__ constexpr int hi(int o) { return K * (o / (2 * K)) + K; }
};

template <typename T, int KIND, int K, int TC>
struct TileArgs {
  using Sh = TileShape<KIND, K, TC>;
  const T* __restrict__ in;
  const T* __restrict__ b;  // operator: r = b - A u if non-null
  T* __restrict__ out;
  int n1_in, n1_out;        // nodes per direction of the input / output grids
  T G0[Sh::NO * Sh::NI];    // M (operator) or the transfer matrix
  T G1[KIND == TILE_OPERATOR ? Sh::NO * Sh::NI : 1];  // K (operator)
};

template <typename T, int KIND, int K, int D, int TC>
struct TileKernelShape {
  using Sh = TileShape<KIND, K, TC>;
  static constexpr int NO = Sh::NO, NI = Sh::NI;
  static constexpr int NT = (KIND == TILE_OPERATOR) ? 2 : 1;  // arrays per stage
  static constexpr int ID2 = (D == 3) ? NI : 1;
  static constexpr int OD2 = (D == 3) ? NO : 1;
  static constexpr int BOX = ID2 * NI * NI;
  static constexpr int XS = NT * ID2 * NI * NO;
  static constexpr int YS = NT * ID2 * NO * NO;  // 3D: after y; 2D: final
  static constexpr int ZS = OD2 * NO * NO;
  static constexpr int BUF0 = (BOX > YS ? BOX : YS);
  static constexpr int BUF1 = (XS > ZS ? XS : ZS);
};

template <typename T, int KIND, int K, int D, int TC>
__global__ void __launch_bounds__(kBlock) tile_kernel(const TileArgs<T, KIND, K, TC> a) {
  using Sh = TileShape<KIND, K, TC>;
  using KS = TileKernelShape<T, KIND, K, D, TC>;
  constexpr int NO = Sh::NO, NI = Sh::NI, NT = KS::NT;
  __shared__ T buf0[KS::BUF0];
  __shared__ T buf1[KS::BUF1];
  const int tid = threadIdx.x;
  int c0[3] = {(int)blockIdx.x * TC, (int)blockIdx.y * TC, (D == 3) ? (int)blockIdx.z * TC : 0};
  // input / output node origins of the tile, per direction
  int in0[3], out0[3];
  for (int e = 0; e < 3; ++e) {
    if (KIND == TILE_OPERATOR) { in0[e] = K * (c0[e] - 1); out0[e] = K * c0[e]; }
    if (KIND == TILE_RESTRICT) { in0[e] = 2 * K * (c0[e] - 1); out0[e] = K * c0[e]; }
    if (KIND == TILE_PROLONG) { in0[e] = K * c0[e]; out0[e] = 2 * K * c0[e]; }
  }
  const int ni = a.n1_in, no = a.n1_out;

  T* box = buf0;
  for (int w = tid; w < KS::BOX; w += kBlock) {
    const int x = w % NI;
    const int y = (w / NI) % NI;
    const int z = w / (NI * NI);
    const int gx = in0[0] + x, gy = in0[1] + y, gz = (D == 3) ? in0[2] + z : 0;
    T v = T(0);
    if (gx >= 0 && gx < ni && gy >= 0 && gy < ni && gz >= 0 && gz < ((D == 3) ? ni : 1))
      v = a.in[(size_t)gx + (size_t)ni * ((size_t)gy + (size_t)ni * (size_t)gz)];
    box[w] = v;
  }
  __syncthreads();

  // x: X[t][z][y][o]
  T* X = buf1;
  constexpr int XA = KS::ID2 * NI * NO;
  for (int w = tid; w < KS::ID2 * NI; w += kBlock) {
    T v[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) v[i] = box[w * NI + i];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        if (i < Sh::lo(o) || i > Sh::hi(o)) continue;
        s0 += a.G0[o * NI + i] * v[i];
        if (NT == 2) s1 += a.G1[o * NI + i] * v[i];
      }
      X[w * NO + o] = s0;
      if (NT == 2) X[XA + w * NO + o] = s1;
    }
  }
  __syncthreads();

  // y: 3D: Y[t][z][o][ox]; 2D: final F[o][ox]
  T* Y = buf0;
  constexpr int YA = KS::ID2 * NO * NO;
  for (int w = tid; w < KS::ID2 * NO; w += kBlock) {
    const int ox = w % NO;
    const int z = w / NO;
    T xm[NI], xk[NI];
#pragma unroll
    for (int y = 0; y < NI; ++y) {
      xm[y] = X[(z * NI + y) * NO + ox];
      if (NT == 2) xk[y] = X[XA + (z * NI + y) * NO + ox];
    }
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int y = 0; y < NI; ++y) {
        if (y < Sh::lo(o) || y > Sh::hi(o)) continue;
        if (NT == 2) {
          if (D == 3) {
            s0 += a.G0[o * NI + y] * xk[y] + a.G1[o * NI + y] * xm[y];
            s1 += a.G0[o * NI + y] * xm[y];
          } else {
            s0 += a.G0[o * NI + y] * xk[y] + a.G1[o * NI + y] * xm[y];
          }
        } else {
          s0 += a.G0[o * NI + y] * xm[y];
        }
      }
      Y[(z * NO + o) * NO + ox] = s0;
      if (NT == 2 && D == 3) Y[YA + (z * NO + o) * NO + ox] = s1;
    }
  }
  __syncthreads();

  T* F = Y;  // final NO^D values (2D)
  if constexpr (D == 3) {
    F = buf1;
    for (int w = tid; w < NO * NO; w += kBlock) {
      T g0[NI], g1[NI];
#pragma unroll
      for (int z = 0; z < NI; ++z) {
        g0[z] = Y[z * NO * NO + w];
        if (NT == 2) g1[z] = Y[YA + z * NO * NO + w];
      }
#pragma unroll
      for (int o = 0; o < NO; ++o) {
        T s = T(0);
#pragma unroll
        for (int z = 0; z < NI; ++z) {
          if (z < Sh::lo(o) || z > Sh::hi(o)) continue;
          if (NT == 2) s += a.G0[o * NI + z] * g0[z] + a.G1[o * NI + z] * g1[z];
          else s += a.G0[o * NI + z] * g0[z];
        }
        F[o * NO * NO + w] = s;
      }
    }
    __syncthreads();
  }

  // write: outputs o in [0, NO] per direction; index NO only for the last grid node
  constexpr int NOE = NO + 1;
  constexpr int NW = (D == 3) ? NOE * NOE * NOE : NOE * NOE;
  for (int w = tid; w < NW; w += kBlock) {
    const int ox = w % NOE;
    const int oy = (w / NOE) % NOE;
    const int oz = (D == 3) ? w / (NOE * NOE) : 0;
    const int gx = out0[0] + ox, gy = out0[1] + oy, gz = (D == 3) ? out0[2] + oz : 0;
    if (gx >= no || gy >= no || gz >= ((D == 3) ? no : 1)) continue;
    if ((ox == NO && gx != no - 1) || (oy == NO && gy != no - 1) || (D == 3 && oz == NO && gz != no - 1)) continue;
    const bool dir = gx == 0 || gx == no - 1 || gy == 0 || gy == no - 1 ||
                     (D == 3 && (gz == 0 || gz == no - 1));
    const size_t g = (size_t)gx + (size_t)no * ((size_t)gy + (size_t)no * (size_t)gz);
    if (KIND == TILE_PROLONG) {
      if (!dir) a.out[g] += F[(oz * NO + oy) * NO + ox];
    } else {
      T v = T(0);
      if (!dir) {
        v = F[(oz * NO + oy) * NO + ox];
        if (KIND == TILE_OPERATOR && a.b != nullptr) v = a.b[g] - v;
      }
      a.out[g] = v;
    }
  }
}

}  // namespace vps
