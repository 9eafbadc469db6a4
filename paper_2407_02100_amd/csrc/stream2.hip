// Row-streaming 2D operator A u (and residual b - A u) for constant
// coefficient, Q_k on a uniform mesh: A = K_x (x) M_y + M_x (x) K_y (the
// Kronecker-sum form of the Laplacian on Cartesian cells, Appendix A.3).
//
// One wavefront owns a strip of 64 - 2K output columns (its lanes cover the
// strip plus K halo columns on each side, one column per lane) and walks a
// chunk of cell rows along y.  Each input row is loaded once as a contiguous
// run, contracted along x from LDS with the lane's row of the banded 1D
// matrices (M_x u, K_x u), and folded into the output rows of its cell with
// the cell matrices in registers; the value on the vertex row shared by two
// cells is carried from one cell to the next, and a row is written once its
// cells have gone by.  A chunk starts one cell early (the carry into its first
// vertex row) and writes its own rows only.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "launch.h"
#include "patch_wave.h"

namespace vps {

namespace {

template <typename T, int K>
struct Op2Args {
  const T* __restrict__ in;
  const T* __restrict__ b;  // out = b - A u if non-null
  T* __restrict__ out;
  int n1, ncell;
  int strips;               // column strips of 64 - 2K output columns
  int cz;                   // cell rows per chunk
  unsigned nblocks;         // strips * chunks
  unsigned vec_bytes;       // bytes of one vector (< 2^32)
  T mc[(K + 1) * (K + 1)];  // cell mass matrix (h-scaled), row-major
  T kc[(K + 1) * (K + 1)];  // cell stiffness matrix
};

template <typename T, int K>
__global__ void __launch_bounds__(64) stream2_operator_kernel(const Op2Args<T, K> a) {
  constexpr int W = K + 1, WO = 64 - 2 * K;
  __shared__ T row[64];

  const unsigned h = blockIdx.x;
  const unsigned per = gridDim.x / kXcd;
  const unsigned logical = (h % kXcd) * per + h / kXcd;
  if (logical >= a.nblocks) return;
  const int lane = threadIdx.x;
  const int strip = (int)(logical % (unsigned)a.strips);
  const int chunk = (int)(logical / (unsigned)a.strips);
  const int c0 = chunk * a.cz, c1 = min(a.ncell, c0 + a.cz);
  const int cs = max(c0 - 1, 0);
  const int n1 = a.n1;
  const int x = strip * WO - K + lane;  // this lane's column (may lie outside the grid)
  const bool xin = x >= 0 && x < n1;
  const bool out_lane = lane >= K && lane < 64 - K && xin;
  const bool xdir = x == 0 || x == n1 - 1;
  const __amdgpu_buffer_rsrc_t ir = make_rsrc(a.in, a.vec_bytes);
  const __amdgpu_buffer_rsrc_t br = make_rsrc(a.b, a.vec_bytes);
  const __amdgpu_buffer_rsrc_t orr = make_rsrc(a.out, a.vec_bytes);
  const unsigned xoff = (unsigned)(xin ? x : 0) * (unsigned)sizeof(T);
  const unsigned srow = (unsigned)n1 * (unsigned)sizeof(T);

  // the lane's row of the assembled 1D matrices, offsets -K..K from its column
  T cmx[2 * K + 1], ckx[2 * K + 1];
  {
    const int al = ((x % K) + K) % K;  // position inside the x cell (0: vertex)
#pragma unroll
    for (int d = -K; d <= K; ++d) {
      T m = T(0), s = T(0);
#pragma unroll
      for (int q = 1; q < K; ++q) {  // inside a cell: one cell matrix row
        if (d + q >= 0 && d + q <= K) {
          m = (al == q) ? a.mc[q * W + d + q] : m;
          s = (al == q) ? a.kc[q * W + d + q] : s;
        }
      }
      T mv, sv;  // a vertex: the two cells it joins
      if (d < 0) { mv = a.mc[K * W + K + d]; sv = a.kc[K * W + K + d]; }
      else if (d > 0) { mv = a.mc[d]; sv = a.kc[d]; }
      else { mv = a.mc[K * W + K] + a.mc[0]; sv = a.kc[K * W + K] + a.kc[0]; }
      cmx[d + K] = (al == 0) ? mv : m;
      ckx[d + K] = (al == 0) ? sv : s;
    }
  }

  // x contraction of input row y: (M_x u, K_x u) at the lane's column
  auto xrow = [&](int y, T& mx, T& kx) {
    const T v = xin ? buf_load<T>(ir, xoff, srow * (unsigned)y) : T(0);
    row[lane] = v;
    __syncthreads();
    mx = T(0);
    kx = T(0);
#pragma unroll
    for (int d = -K; d <= K; ++d) {
      const int l = min(max(lane + d, 0), 63);
      const T w = row[l];
      mx = fma(cmx[d + K], w, mx);
      kx = fma(ckx[d + K], w, kx);
    }
    __syncthreads();
  };
  auto emit = [&](int y, T v) {
    if (!out_lane) return;
    const bool dir = xdir || y == 0 || y == n1 - 1;
    T o = T(0);
    if (!dir) o = a.b ? buf_load<T>(br, xoff, srow * (unsigned)y) - v : v;
    buf_store<T>(o, orr, xoff, srow * (unsigned)y);
  };

  T mx[W], kx[W];
  xrow(K * cs, mx[0], kx[0]);
  T carry = T(0);
  for (int c = cs; c < c1; ++c) {
#pragma unroll
    for (int j = 1; j <= K; ++j) xrow(K * c + j, mx[j], kx[j]);
    T acc[W];
#pragma unroll
    for (int i = 0; i <= K; ++i) {
      T s = T(0);
#pragma unroll
      for (int j = 0; j <= K; ++j) {
        s = fma(a.mc[i * W + j], kx[j], s);
        s = fma(a.kc[i * W + j], mx[j], s);
      }
      acc[i] = s;
    }
    acc[0] += carry;
    if (c >= c0) {
#pragma unroll
      for (int i = 0; i < K; ++i) emit(K * c + i, acc[i]);
    }
    carry = acc[K];
    mx[0] = mx[K];
    kx[0] = kx[K];
  }
  if (c1 == a.ncell) emit(n1 - 1, carry);  // the last grid row (Dirichlet: zero)
}

// ---- restriction r_c = R r_f, R = P^T (1D factors along x and y) ----
//
// One wavefront owns a strip of 64 - 2K coarse output columns (one lane per
// coarse column, K halo lanes on each side; a lane loads the two fine values
// 2X and 2X + 1, so a fine row arrives as one contiguous run of 128 values)
// and walks a chunk of coarse cell rows: the 2K fine rows of a coarse cell
// are contracted along x from LDS with the lane's row of R and folded into
// the cell's K + 1 coarse rows; the coarse vertex row shared by two cells is
// carried.  A chunk starts one coarse cell early (the carry into its first
// vertex row) and writes its own rows only.

template <typename T, int K>
struct Tr2Args {
  const T* __restrict__ in;
  T* __restrict__ out;
  int n1f, n1c, ncc;         // fine and coarse nodes per direction, coarse cells
  int strips, cz;            // column strips, coarse cell rows per chunk
  unsigned nblocks;
  unsigned bytes_in, bytes_out;
  T g[K * (4 * K + 1)];      // restriction: R row of a coarse node at position a (0..K-1) over 4K+1 fine nodes
  T z[(K + 1) * (2 * K + 1)];  // restriction: cell block [coarse i][fine l]; prolongation: P rows [fine j][coarse i]
};

template <typename T, int K>
__global__ void __launch_bounds__(64) stream2_restrict_kernel(const Tr2Args<T, K> a) {
  constexpr int GW = 4 * K + 1, ZW = 2 * K + 1, WO = 64 - 2 * K;
  __shared__ T row[128];
  const unsigned h = blockIdx.x;
  const unsigned per = gridDim.x / kXcd;
  const unsigned logical = (h % kXcd) * per + h / kXcd;
  if (logical >= a.nblocks) return;
  const int lane = threadIdx.x;
  const int strip = (int)(logical % (unsigned)a.strips);
  const int chunk = (int)(logical / (unsigned)a.strips);
  const int c0 = chunk * a.cz, c1 = min(a.ncc, c0 + a.cz);
  const int cs = max(c0 - 1, 0);
  const int X = strip * WO - K + lane;  // this lane's coarse column
  const bool out_lane = lane >= K && lane < 64 - K && X >= 0 && X < a.n1c;
  const bool xdir = X == 0 || X == a.n1c - 1;
  const __amdgpu_buffer_rsrc_t ir = make_rsrc(a.in, a.bytes_in);
  const __amdgpu_buffer_rsrc_t orr = make_rsrc(a.out, a.bytes_out);
  const int f0 = 2 * X, f1 = 2 * X + 1;  // the two fine columns this lane loads
  const bool in0 = f0 >= 0 && f0 < a.n1f, in1 = f1 >= 0 && f1 < a.n1f;
  const unsigned off0 = (unsigned)(in0 ? f0 : 0) * (unsigned)sizeof(T);
  const unsigned off1 = (unsigned)(in1 ? f1 : 0) * (unsigned)sizeof(T);
  const unsigned srf = (unsigned)a.n1f * (unsigned)sizeof(T), src = (unsigned)a.n1c * (unsigned)sizeof(T);
  const unsigned xoff = (unsigned)(out_lane ? X : 0) * (unsigned)sizeof(T);

  // the lane's row of R over fine offsets -2K..2K from 2X
  T cg[GW];
  {
    const int al = ((X % K) + K) % K;
#pragma unroll
    for (int d = -2 * K; d <= 2 * K; ++d) {
      T v = T(0);
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const int i = d + 2 * K + 2 * q;  // index into the 4K+1 window of position q
        if (i >= 0 && i < GW) v = (al == q) ? a.g[q * GW + i] : v;
      }
      cg[d + 2 * K] = v;
    }
  }
  auto xrow = [&](int y) {
    const T v0 = in0 ? buf_load<T>(ir, off0, srf * (unsigned)y) : T(0);
    const T v1 = in1 ? buf_load<T>(ir, off1, srf * (unsigned)y) : T(0);
    row[2 * lane] = v0;
    row[2 * lane + 1] = v1;
    __syncthreads();
    T s = T(0);
#pragma unroll
    for (int d = -2 * K; d <= 2 * K; ++d) s = fma(cg[d + 2 * K], row[min(max(2 * lane + d, 0), 127)], s);
    __syncthreads();
    return s;
  };
  auto emit = [&](int Y, T v) {
    if (!out_lane) return;
    const bool dir = xdir || Y == 0 || Y == a.n1c - 1;
    buf_store<T>(dir ? T(0) : v, orr, xoff, src * (unsigned)Y);
  };
  T carry = T(0);
  for (int c = cs; c < c1; ++c) {
    T acc[K + 1];
#pragma unroll
    for (int i = 0; i <= K; ++i) acc[i] = T(0);
#pragma unroll
    for (int l = 0; l < 2 * K; ++l) {
      const T sx = xrow(2 * K * c + l);
#pragma unroll
      for (int i = 0; i <= K; ++i) acc[i] = fma(a.z[i * ZW + l], sx, acc[i]);
    }
    acc[0] += carry;
    if (c >= c0) {
#pragma unroll
      for (int i = 0; i < K; ++i) emit(K * c + i, acc[i]);
    }
    carry = acc[K];
  }
  if (c1 == a.ncc) emit(a.n1c - 1, carry);  // the last coarse row (Dirichlet: zero)
}

// ---- prolongate-add u_f += P e_c ----
//
// One wavefront owns a strip of 64 fine output columns and walks a chunk of
// coarse cell rows: the K + 1 coarse rows of a cell are contracted along x
// from LDS (each fine column from the K + 1 coarse nodes of its coarse cell)
// and interpolated into the cell's 2K fine rows, which are read, added to and
// written once; the coarse vertex row is shared with the next cell.  Fine
// Dirichlet rows and columns are left as they are.
template <typename T, int K>
__global__ void __launch_bounds__(64) stream2_prolong_kernel(const Tr2Args<T, K> a) {
  constexpr int W = K + 1, S = 2 * K;
  __shared__ T row[64];
  const unsigned h = blockIdx.x;
  const unsigned per = gridDim.x / kXcd;
  const unsigned logical = (h % kXcd) * per + h / kXcd;
  if (logical >= a.nblocks) return;
  const int lane = threadIdx.x;
  const int strip = (int)(logical % (unsigned)a.strips);
  const int chunk = (int)(logical / (unsigned)a.strips);
  const int c0 = chunk * a.cz, c1 = min(a.ncc, c0 + a.cz);
  const int x = strip * 64 + lane;  // this lane's fine column
  const bool xin = x > 0 && x < a.n1f - 1;
  const int cx = min(x, a.n1f - 2) / S;  // its coarse cell
  const int j = min(x, a.n1f - 2) - S * cx;  // its position in the cell (0..2K-1)
  const int X0 = (strip * 64) / S * K;       // first coarse column the strip reads
  const int XL = K * cx - X0;                // this lane's first coarse node, in the strip's coarse row
  const __amdgpu_buffer_rsrc_t ir = make_rsrc(a.in, a.bytes_in);
  const __amdgpu_buffer_rsrc_t orr = make_rsrc(a.out, a.bytes_out);
  const unsigned srf = (unsigned)a.n1f * (unsigned)sizeof(T), src = (unsigned)a.n1c * (unsigned)sizeof(T);
  const int Xl = X0 + lane;  // coarse column loaded by this lane
  const bool cin = Xl < a.n1c;
  const unsigned coff = (unsigned)(cin ? Xl : 0) * (unsigned)sizeof(T);
  const unsigned xoff = (unsigned)(xin ? x : 0) * (unsigned)sizeof(T);
  T pj[W];  // the lane's row of P inside its coarse cell
#pragma unroll
  for (int i = 0; i < W; ++i) {
    T v = T(0);
#pragma unroll
    for (int q = 0; q < S; ++q) v = (j == q) ? a.z[q * W + i] : v;
    pj[i] = v;
  }
  auto xrow = [&](int Y) {
    row[lane] = cin ? buf_load<T>(ir, coff, src * (unsigned)Y) : T(0);
    __syncthreads();
    T s = T(0);
#pragma unroll
    for (int i = 0; i < W; ++i) s = fma(pj[i], row[min(max(XL + i, 0), 63)], s);
    __syncthreads();
    return s;
  };
  T ex[W];
  ex[0] = xrow(K * c0);
  for (int c = c0; c < c1; ++c) {
#pragma unroll
    for (int i = 1; i <= K; ++i) ex[i] = xrow(K * c + i);
#pragma unroll
    for (int q = 0; q < S; ++q) {
      const int y = S * c + q;
      T v = T(0);
#pragma unroll
      for (int i = 0; i < W; ++i) v = fma(a.z[q * W + i], ex[i], v);
      if (xin && y > 0) {
        const T uf = buf_load<T>(orr, xoff, srf * (unsigned)y);
        buf_store<T>(uf + v, orr, xoff, srf * (unsigned)y);
      }
    }
    ex[0] = ex[K];
  }
}

}  // namespace

template <typename T, int K>
hipError_t launch_stream2_operator(const Stream2Launch& L, hipStream_t s) {
  static_assert(sizeof(Op2Args<T, K>) <= 4096, "kernel arguments exceed 4 KiB");
  constexpr int W = K + 1, WO = 64 - 2 * K;
  Op2Args<T, K> a;
  a.in = (const T*)L.in;
  a.b = (const T*)L.b;
  a.out = (T*)L.out;
  a.n1 = L.n1;
  a.ncell = L.ncell;
  a.strips = (L.n1 + WO - 1) / WO;
  // cell rows per chunk: about 8192 wavefronts over the grid, at least 4 cells
  const long long want = std::max(1LL, (long long)a.strips * L.ncell / 8192);
  a.cz = (int)std::min<long long>(L.ncell, std::max<long long>(4, want));
  const long long chunks = (L.ncell + a.cz - 1) / a.cz;
  const unsigned long long nb = (unsigned long long)a.strips * chunks;
  const unsigned long long vbytes = (unsigned long long)L.n1 * L.n1 * sizeof(T);
  if (nb >= (1ull << 31) || vbytes >= (1ull << 32)) return hipErrorInvalidValue;
  a.nblocks = (unsigned)nb;
  a.vec_bytes = (unsigned)vbytes;
  for (int i = 0; i < W * W; ++i) {
    a.mc[i] = (T)L.Mc[i];
    a.kc[i] = (T)L.Kc[i];
  }
  const unsigned grid = (a.nblocks + kXcd - 1) / kXcd * kXcd;  // a multiple of the XCD count
  stream2_operator_kernel<T, K><<<grid, 64, 0, s>>>(a);
  return hipGetLastError();
}

template <typename T, int K>
hipError_t launch_stream2_restrict(const Stream2Launch& L, hipStream_t s) {
  static_assert(sizeof(Tr2Args<T, K>) <= 4096, "kernel arguments exceed 4 KiB");
  constexpr int WO = 64 - 2 * K;
  Tr2Args<T, K> a;
  a.in = (const T*)L.in;
  a.out = (T*)L.out;
  a.ncc = L.ncell;  // coarse cells
  a.n1c = K * L.ncell + 1;
  a.n1f = 2 * K * L.ncell + 1;
  a.strips = (a.n1c + WO - 1) / WO;
  const long long want = std::max(1LL, (long long)a.strips * a.ncc / 8192);
  a.cz = (int)std::min<long long>(a.ncc, std::max<long long>(4, want));
  const long long chunks = (a.ncc + a.cz - 1) / a.cz;
  const unsigned long long nb = (unsigned long long)a.strips * chunks;
  const unsigned long long bi = (unsigned long long)a.n1f * a.n1f * sizeof(T);
  const unsigned long long bo = (unsigned long long)a.n1c * a.n1c * sizeof(T);
  if (nb >= (1ull << 31) || bi >= (1ull << 32)) return hipErrorInvalidValue;
  a.nblocks = (unsigned)nb;
  a.bytes_in = (unsigned)bi;
  a.bytes_out = (unsigned)bo;
  for (int i = 0; i < K * (4 * K + 1); ++i) a.g[i] = (T)L.Mc[i];
  for (int i = 0; i < (K + 1) * (2 * K + 1); ++i) a.z[i] = (T)L.Kc[i];
  const unsigned grid = (a.nblocks + kXcd - 1) / kXcd * kXcd;
  stream2_restrict_kernel<T, K><<<grid, 64, 0, s>>>(a);
  return hipGetLastError();
}

template <typename T, int K>
hipError_t launch_stream2_prolong(const Stream2Launch& L, hipStream_t s) {
  static_assert(sizeof(Tr2Args<T, K>) <= 4096, "kernel arguments exceed 4 KiB");
  Tr2Args<T, K> a;
  a.in = (const T*)L.in;
  a.out = (T*)L.out;
  a.ncc = L.ncell;
  a.n1c = K * L.ncell + 1;
  a.n1f = 2 * K * L.ncell + 1;
  a.strips = (a.n1f + 63) / 64;
  const long long want = std::max(1LL, (long long)a.strips * a.ncc / 8192);
  a.cz = (int)std::min<long long>(a.ncc, std::max<long long>(4, want));
  const long long chunks = (a.ncc + a.cz - 1) / a.cz;
  const unsigned long long nb = (unsigned long long)a.strips * chunks;
  const unsigned long long bi = (unsigned long long)a.n1c * a.n1c * sizeof(T);
  const unsigned long long bo = (unsigned long long)a.n1f * a.n1f * sizeof(T);
  if (nb >= (1ull << 31) || bo >= (1ull << 32)) return hipErrorInvalidValue;
  a.nblocks = (unsigned)nb;
  a.bytes_in = (unsigned)bi;
  a.bytes_out = (unsigned)bo;
  for (int i = 0; i < K * (4 * K + 1); ++i) a.g[i] = T(0);
  for (int i = 0; i < 2 * K * (K + 1); ++i) a.z[i] = (T)L.Mc[i];
  const unsigned grid = (a.nblocks + kXcd - 1) / kXcd * kXcd;
  stream2_prolong_kernel<T, K><<<grid, 64, 0, s>>>(a);
  return hipGetLastError();
}

#define VPS_STREAM2(T, K)                                                             \
  template hipError_t launch_stream2_operator<T, K>(const Stream2Launch&, hipStream_t); \
  template hipError_t launch_stream2_restrict<T, K>(const Stream2Launch&, hipStream_t); \
  template hipError_t launch_stream2_prolong<T, K>(const Stream2Launch&, hipStream_t);
VPS_STREAM2(double, 1)
VPS_STREAM2(double, 2)
VPS_STREAM2(double, 3)
VPS_STREAM2(double, 4)
VPS_STREAM2(double, 5)
VPS_STREAM2(float, 1)
VPS_STREAM2(float, 2)
VPS_STREAM2(float, 3)
VPS_STREAM2(float, 4)
VPS_STREAM2(float, 5)
#undef VPS_STREAM2

}  // namespace vps
