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

#define VPS_STREAM2(T, K) template hipError_t launch_stream2_operator<T, K>(const Stream2Launch&, hipStream_t);
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
