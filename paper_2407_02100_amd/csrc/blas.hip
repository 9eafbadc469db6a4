// Vector kernels, coarse solvers and coefficient coarsening of libvps.
#include "kernels.h"
#include "launch.h"

namespace vps {

namespace {

inline unsigned grid_for(size_t n) {
  size_t g = (n + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  if (g == 0) g = 1;
  return (unsigned)g;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) fill_kernel(T* __restrict__ x, T v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) x[i] = v;
}

template <typename Ti, typename To>
__global__ void __launch_bounds__(kBlock) cast_kernel(const Ti* __restrict__ in, To* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
    out[i] = (To)in[i];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) axpy_kernel(T a, const T* __restrict__ x, T* __restrict__ y, size_t n) {
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
    y[i] += a * x[i];
}

__global__ void __launch_bounds__(kBlock) xpay_kernel(const double* __restrict__ x, double a, double* __restrict__ y,
                                                      size_t n) {
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
    y[i] = x[i] + a * y[i];
}

// Deterministic block reduction of one double per thread.
__device__ inline double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

// x += alpha p (x = alpha p when x_zero), r = r_in - alpha q, optionally r32 = (float) r,
// partial sums of r.r
__global__ void __launch_bounds__(kBlock) cg_update_kernel(double alpha, const double* __restrict__ p,
                                                           const double* __restrict__ q, double* __restrict__ x,
                                                           const double* r_in, double* r, float* __restrict__ r32,
                                                           bool x_zero, size_t n, double* __restrict__ partial) {
  __shared__ double red[kBlock];
  double acc = 0.0;
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    x[i] = x_zero ? alpha * p[i] : x[i] + alpha * p[i];
    const double ri = r_in[i] - alpha * q[i];
    r[i] = ri;
    if (r32) r32[i] = (float)ri;
    acc += ri * ri;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// partial sums of (r.z) and, if q is given, (z.q), with z in FP32
__global__ void __launch_bounds__(kBlock) dot_z32_kernel(const double* __restrict__ r, const float* __restrict__ z,
                                                         const double* __restrict__ q, size_t n,
                                                         double* __restrict__ partial) {
  __shared__ double red[kBlock];
  double a1 = 0.0, a2 = 0.0;
  const bool two = q != nullptr;
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    const double zi = (double)z[i];
    a1 += r[i] * zi;
    if (two) a2 += zi * q[i];
  }
  const double s1 = block_sum(a1, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s1;
  if (two) {
    const double s2 = block_sum(a2, red);
    if (threadIdx.x == 0) partial[gridDim.x + blockIdx.x] = s2;
  }
}

// p = (double) z + beta p
__global__ void __launch_bounds__(kBlock) xpay_z32_kernel(const float* __restrict__ z, double beta,
                                                          double* __restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
    p[i] = (double)z[i] + beta * p[i];
}

__global__ void __launch_bounds__(kBlock) dot_partial_kernel(const double* __restrict__ x,
                                                             const double* __restrict__ y,
                                                             const double* __restrict__ x2,
                                                             const double* __restrict__ y2, size_t n,
                                                             double* __restrict__ partial) {
  __shared__ double red[kBlock];
  double a1 = 0.0, a2 = 0.0;
  const bool two = x2 != nullptr;
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    a1 += x[i] * y[i];
    if (two) a2 += x2[i] * y2[i];
  }
  const double s1 = block_sum(a1, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s1;
  if (two) {
    const double s2 = block_sum(a2, red);
    if (threadIdx.x == 0) partial[gridDim.x + blockIdx.x] = s2;
  }
}

__global__ void __launch_bounds__(kBlock) dot_final_kernel(const double* __restrict__ partial, int nblk,
                                                           double* __restrict__ out) {
  __shared__ double red[kBlock];
  const double* p = partial + (size_t)blockIdx.x * nblk;
  double a = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kBlock) a += p[i];
  const double s = block_sum(a, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock) coarsen_rho_kernel(const double* __restrict__ fine,
                                                             double* __restrict__ coarse, int nc, int D) {
  const size_t total = (D == 3) ? (size_t)nc * nc * nc : (size_t)nc * nc;
  const int nf = 2 * nc;
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < total; i += (size_t)gridDim.x * kBlock) {
    const int cx = (int)(i % nc);
    const int cy = (int)((i / nc) % nc);
    const int cz = (D == 3) ? (int)(i / ((size_t)nc * nc)) : 0;
    double s = 0.0;
    for (int c = 0; c < (1 << D); ++c) {
      const int fx = 2 * cx + (c & 1), fy = 2 * cy + ((c >> 1) & 1), fz = (D == 3) ? 2 * cz + ((c >> 2) & 1) : 0;
      s += fine[(size_t)fx + (size_t)nf * ((size_t)fy + (size_t)nf * (size_t)fz)];
    }
    coarse[i] = s / (double)(1 << D);
  }
}

// ---- coarse solve by fast diagonalisation of the whole coarse grid ----
template <typename T, int D>
struct CoarseArgs {
  static constexpr int NMAX = (D == 3) ? 15 : 63;
  const T* __restrict__ b;
  T* __restrict__ x;
  const T* __restrict__ T0;   // n0 x n0 (device)
  const T* __restrict__ lam;  // n0 (device)
  int n0;
};

// one line transform along direction `dir` of an n0^D box: out = op(in)
// transpose=true: out[m] = sum_i T[i][m] in[i]; else out[i] = sum_m T[i][m] in[m].
// A work item computes one output of one line (the items of a line share
// their reads of `in`); Tm is in LDS in 3D.
constexpr int kCoarseBlock = 1024;

template <typename T, int D>
__device__ void coarse_lines(const T* Tm, int n, const T* in, T* out, int dir, bool transpose) {
  const int nlines = (D == 3) ? n * n : n;
  const int stride = (dir == 0) ? 1 : (dir == 1 ? n : n * n);
  for (int w = threadIdx.x; w < nlines * n; w += kCoarseBlock) {
    const int line = w / n, o = w % n;
    int base;
    if (dir == 0) base = line * n;
    else if (dir == 1) base = (D == 3) ? (line / n) * n * n + (line % n) : line;
    else base = line;
    T s = T(0);
    for (int i = 0; i < n; ++i) s += (transpose ? Tm[i * n + o] : Tm[o * n + i]) * in[base + i * stride];
    out[base + o * stride] = s;
  }
}

template <typename T, int D>
__global__ void __launch_bounds__(kCoarseBlock) coarse_fdm_kernel(const CoarseArgs<T, D> a) {
  constexpr int NMAX = CoarseArgs<T, D>::NMAX;
  constexpr int SZ = (D == 3) ? NMAX * NMAX * NMAX : NMAX * NMAX;
  __shared__ T A[SZ];
  __shared__ T B[SZ];
  __shared__ T TS[(D == 3) ? NMAX * NMAX : 1];
  const int n = a.n0, n1 = n + 2;
  const int tot = (D == 3) ? n * n * n : n * n;
  const T* Tm = a.T0;  // 2D: the matrix stays in global memory (A and B fill the LDS)
  if constexpr (D == 3) {
    for (int w = threadIdx.x; w < n * n; w += kCoarseBlock) TS[w] = a.T0[w];
    Tm = TS;
  }
  for (int w = threadIdx.x; w < tot; w += kCoarseBlock) {
    const int x = w % n, y = (w / n) % n, z = (D == 3) ? w / (n * n) : -1;
    A[w] = a.b[(size_t)(x + 1) + (size_t)n1 * ((size_t)(y + 1) + (size_t)n1 * (size_t)(z + 1))];
  }
  __syncthreads();
  coarse_lines<T, D>(Tm, n, A, B, 0, true);
  __syncthreads();
  coarse_lines<T, D>(Tm, n, B, A, 1, true);
  __syncthreads();
  T* cur = A;
  T* oth = B;
  if (D == 3) {
    coarse_lines<T, D>(Tm, n, A, B, 2, true);
    __syncthreads();
    cur = B;
    oth = A;
  }
  for (int w = threadIdx.x; w < tot; w += kCoarseBlock) {
    const int x = w % n, y = (w / n) % n, z = (D == 3) ? w / (n * n) : 0;
    T l = a.lam[x] + a.lam[y];
    if (D == 3) l += a.lam[z];
    cur[w] = cur[w] / l;
  }
  __syncthreads();
  if (D == 3) {
    coarse_lines<T, D>(Tm, n, cur, oth, 2, false);
    __syncthreads();
    T* t = cur; cur = oth; oth = t;
  }
  coarse_lines<T, D>(Tm, n, cur, oth, 1, false);
  __syncthreads();
  coarse_lines<T, D>(Tm, n, oth, cur, 0, false);
  __syncthreads();
  const int all = (D == 3) ? n1 * n1 * n1 : n1 * n1;
  for (int w = threadIdx.x; w < all; w += kCoarseBlock) {
    const int x = w % n1, y = (w / n1) % n1, z = (D == 3) ? w / (n1 * n1) : 1;
    const bool inside = x > 0 && x < n1 - 1 && y > 0 && y < n1 - 1 && (D == 2 || (z > 0 && z < n1 - 1));
    a.x[w] = inside ? cur[(x - 1) + n * ((y - 1) + n * (D == 3 ? z - 1 : 0))] : T(0);
  }
}

// ---- coarse solve with an explicit dense inverse (one wave per row) ----
template <typename T>
__global__ void __launch_bounds__(kBlock) coarse_dense_kernel(const T* __restrict__ Ainv, const int* __restrict__ fidx,
                                                              int nf, const T* __restrict__ b, T* __restrict__ x) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (row >= nf) return;
  T s = T(0);
  const T* Ar = Ainv + (size_t)row * nf;
  for (int c = lane; c < nf; c += 64) s += Ar[c] * b[fidx[c]];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) x[fidx[row]] = s;
}

}  // namespace

template <typename T>
hipError_t launch_fill(void* x, double v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  fill_kernel<T><<<grid_for(n), kBlock, 0, s>>>((T*)x, (T)v, n);
  return hipGetLastError();
}
template hipError_t launch_fill<double>(void*, double, size_t, hipStream_t);
template hipError_t launch_fill<float>(void*, double, size_t, hipStream_t);

template <typename Ti, typename To>
hipError_t launch_cast(const void* in, void* out, size_t n, hipStream_t s) {
  cast_kernel<Ti, To><<<grid_for(n), kBlock, 0, s>>>((const Ti*)in, (To*)out, n);
  return hipGetLastError();
}
template hipError_t launch_cast<double, float>(const void*, void*, size_t, hipStream_t);
template hipError_t launch_cast<float, double>(const void*, void*, size_t, hipStream_t);
template hipError_t launch_cast<double, double>(const void*, void*, size_t, hipStream_t);
template hipError_t launch_cast<float, float>(const void*, void*, size_t, hipStream_t);

template <typename T>
hipError_t launch_axpy(double a, const void* x, void* y, size_t n, hipStream_t s) {
  axpy_kernel<T><<<grid_for(n), kBlock, 0, s>>>((T)a, (const T*)x, (T*)y, n);
  return hipGetLastError();
}
template hipError_t launch_axpy<double>(double, const void*, void*, size_t, hipStream_t);
template hipError_t launch_axpy<float>(double, const void*, void*, size_t, hipStream_t);

hipError_t launch_xpay(const double* x, double a, double* y, size_t n, hipStream_t s) {
  xpay_kernel<<<grid_for(n), kBlock, 0, s>>>(x, a, y, n);
  return hipGetLastError();
}

static int dot_blocks(size_t n) {
  size_t g = (n + kBlock - 1) / kBlock;
  if (g > (size_t)kDotBlocks) g = kDotBlocks;
  if (g == 0) g = 1;
  return (int)g;
}

hipError_t launch_cg_update(double alpha, const double* p, const double* q, double* x, const double* r_in,
                            double* r, float* r32, bool x_zero, size_t n, double* partial, int* nblk,
                            hipStream_t s) {
  const int g = dot_blocks(n);
  *nblk = g;
  cg_update_kernel<<<g, kBlock, 0, s>>>(alpha, p, q, x, r_in, r, r32, x_zero, n, partial);
  return hipGetLastError();
}

hipError_t launch_dot_z32(const double* r, const float* z, const double* q, size_t n, double* partial, int* nblk,
                          hipStream_t s) {
  const int g = dot_blocks(n);
  *nblk = g;
  dot_z32_kernel<<<g, kBlock, 0, s>>>(r, z, q, n, partial);
  return hipGetLastError();
}

hipError_t launch_xpay_z32(const float* z, double beta, double* p, size_t n, hipStream_t s) {
  xpay_z32_kernel<<<grid_for(n), kBlock, 0, s>>>(z, beta, p, n);
  return hipGetLastError();
}

hipError_t launch_dot_partial(const double* x, const double* y, const double* x2, const double* y2, size_t n,
                              double* partial, int* nblk, hipStream_t s) {
  const int g = dot_blocks(n);
  *nblk = g;
  dot_partial_kernel<<<g, kBlock, 0, s>>>(x, y, x2, y2, n, partial);
  return hipGetLastError();
}

hipError_t launch_dot_final(const double* partial, int nblk, int ndot, double* out, hipStream_t s) {
  dot_final_kernel<<<ndot, kBlock, 0, s>>>(partial, nblk, out);
  return hipGetLastError();
}

hipError_t launch_coarsen_rho(const double* fine, double* coarse, int ncell_coarse, int D, hipStream_t s) {
  const size_t total = (D == 3) ? (size_t)ncell_coarse * ncell_coarse * ncell_coarse
                                : (size_t)ncell_coarse * ncell_coarse;
  coarsen_rho_kernel<<<grid_for(total), kBlock, 0, s>>>(fine, coarse, ncell_coarse, D);
  return hipGetLastError();
}

template <typename T, int D>
hipError_t launch_coarse_fdm(const CoarseFdmLaunch& L, hipStream_t s) {
  CoarseArgs<T, D> a;
  a.b = (const T*)L.b;
  a.x = (T*)L.x;
  a.n0 = L.n0;
  a.T0 = (const T*)L.T0;
  a.lam = (const T*)L.lam0;
  if (L.n0 > CoarseArgs<T, D>::NMAX || L.n0 < 1) return hipErrorInvalidValue;
  coarse_fdm_kernel<T, D><<<1, kCoarseBlock, 0, s>>>(a);
  return hipGetLastError();
}
template hipError_t launch_coarse_fdm<double, 2>(const CoarseFdmLaunch&, hipStream_t);
template hipError_t launch_coarse_fdm<double, 3>(const CoarseFdmLaunch&, hipStream_t);
template hipError_t launch_coarse_fdm<float, 2>(const CoarseFdmLaunch&, hipStream_t);
template hipError_t launch_coarse_fdm<float, 3>(const CoarseFdmLaunch&, hipStream_t);

template <typename T>
hipError_t launch_coarse_dense(const void* Ainv, const int* free_idx, int nfree, const void* b, void* x,
                               size_t nodes, hipStream_t s) {
  hipError_t e = launch_fill<T>(x, 0.0, nodes, s);
  if (e != hipSuccess) return e;
  const int rows_per_block = kBlock / 64;
  coarse_dense_kernel<T><<<(nfree + rows_per_block - 1) / rows_per_block, kBlock, 0, s>>>(
      (const T*)Ainv, free_idx, nfree, (const T*)b, (T*)x);
  return hipGetLastError();
}
template hipError_t launch_coarse_dense<double>(const void*, const int*, int, const void*, void*, size_t,
                                                hipStream_t);
template hipError_t launch_coarse_dense<float>(const void*, const int*, int, const void*, void*, size_t,
                                               hipStream_t);

}  // namespace vps
