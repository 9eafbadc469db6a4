// Solve-only patch kernel for the separated colorized smoother (Algorithm 3):
// u_int += A_j^{-1} r_int for every patch of one color, with r = b - A u the
// global residual computed before the color by the operator kernel.  3D,
// constant coefficient, one patch per wavefront, fast diagonalization in the
// even/odd form of the combined kernel.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "patch_wave.h"

namespace vps {

template <typename T, int K>
struct SolveArgs {
  T* __restrict__ u;
  const T* __restrict__ r;
  int n1;
  int v0[3];
  int np[3];
  unsigned npatch;
  unsigned vec_bytes;  // bytes of one level vector (< 2^32)
  unsigned magic_x, magic_y;  // magic_of(np[0]), magic_of(np[1]) (see div_magic)
  WaveFdm<T, K> f;
  T lam[2 * K - 1];  // 1D generalized eigenvalues in the internal mode order
};

// v[i] for a lane-dependent i < N, from kernel-argument values
template <typename T, int N>
__device__ inline T pick_lane(const T (&v)[N], int i) {
  T out = v[0];
#pragma unroll
  for (int j = 1; j < N; ++j) out = (i == j) ? v[j] : out;
  return out;
}

// Lanes of the wave that owns a patch (Q^2 <= 64 lanes active):
//   A. r and u interior columns (y, x) along z, T^T along z in registers;
//   B. T^T along x;  C. T^T along y, 1/Lambda, T along y;  D. T along x;
//   E. T along z, u_int + d stored plane by plane.
template <typename T, int K>
__global__ void __launch_bounds__(64) patch_solve3_kernel(const SolveArgs<T, K> a) {
  constexpr int Q = 2 * K - 1, Q2 = Q * Q;
  static_assert(Q2 <= 64, "one wave per patch needs (2K-1)^2 <= 64");
  __shared__ T W0[Q * Q2];
  __shared__ T W1[Q * Q2];

  const unsigned h = blockIdx.x;
  const unsigned per = gridDim.x / kXcd;
  const unsigned logical = (h % kXcd) * per + h / kXcd;
  if (logical >= a.npatch) return;
  const int lane = threadIdx.x;
  const unsigned npx = (unsigned)a.np[0], npy = (unsigned)a.np[1];
  const unsigned qx = div_magic(logical, npx, a.magic_x);
  const unsigned qy = div_magic(qx, npy, a.magic_y);
  const int px = (int)(logical - qx * npx);
  const int py = (int)(qx - qy * npy);
  const int pz = (int)qy;
  const unsigned n1 = (unsigned)a.n1;
  const size_t n2 = (size_t)n1 * n1;
  // first interior node of the patch
  const size_t base = (size_t)(K * (a.v0[0] + 2 * px - 1) + 1) + (size_t)n1 * (size_t)(K * (a.v0[1] + 2 * py - 1) + 1) +
                      n2 * (size_t)(K * (a.v0[2] + 2 * pz - 1) + 1);
  const __amdgpu_buffer_rsrc_t ur = make_rsrc(a.u, a.vec_bytes);
  const __amdgpu_buffer_rsrc_t rr = make_rsrc(a.r, a.vec_bytes);
  const unsigned sbase = (unsigned)(base * sizeof(T));
  const unsigned splane = (unsigned)(n2 * sizeof(T));
  const int ly = lane / Q, lx = lane % Q;  // (y, x) in stages A and E; (mode z, y or mode x) in B-D

  // ---- A. loads, T^T along z ----
  T uc[Q];
  if (lane < Q2) {
    const unsigned off = (n1 * (unsigned)ly + (unsigned)lx) * (unsigned)sizeof(T);
    T rc[Q], m[Q];
#pragma unroll
    for (int z = 0; z < Q; ++z) {
      rc[z] = buf_load<T>(rr, off, sbase + splane * z);
      uc[z] = buf_load<T>(ur, off, sbase + splane * z);
    }
    fdm_forward<T, K>(a.f, rc, m);
#pragma unroll
    for (int j = 0; j < Q; ++j) W0[(j * Q + ly) * Q + lx] = m[j];
  }
  __syncthreads();
  // ---- B. T^T along x  (lanes (mz, y)) ----
  if (lane < Q2) {
    T v[Q], m[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = W0[(ly * Q + lx) * Q + i];
    fdm_forward<T, K>(a.f, v, m);
#pragma unroll
    for (int j = 0; j < Q; ++j) W1[(ly * Q + lx) * Q + j] = m[j];
  }
  __syncthreads();
  // ---- C. T^T along y, 1/Lambda, T along y  (lanes (mz, mx)) ----
  if (lane < Q2) {
    T v[Q], c[Q], d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = W1[(ly * Q + i) * Q + lx];
    fdm_forward<T, K>(a.f, v, c);
    const T s2 = pick_lane<T, Q>(a.lam, ly) + pick_lane<T, Q>(a.lam, lx);
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      c[j] *= inv_eig(s2 + a.lam[j]);
    }
    fdm_backward<T, K>(a.f, c, d);
#pragma unroll
    for (int i = 0; i < Q; ++i) W0[(ly * Q + i) * Q + lx] = d[i];
  }
  __syncthreads();
  // ---- D. T along x  (lanes (mz, y)) ----
  if (lane < Q2) {
    T c[Q], d[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) c[j] = W0[(ly * Q + lx) * Q + j];
    fdm_backward<T, K>(a.f, c, d);
#pragma unroll
    for (int i = 0; i < Q; ++i) W1[(ly * Q + lx) * Q + i] = d[i];
  }
  __syncthreads();
  // ---- E. T along z, update, store  (lanes (y, x)) ----
  if (lane < Q2) {
    T c[Q], d[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) c[j] = W1[(j * Q + ly) * Q + lx];
    fdm_backward<T, K>(a.f, c, d);
    const unsigned off = (n1 * (unsigned)ly + (unsigned)lx) * (unsigned)sizeof(T);
#pragma unroll
    for (int z = 0; z < Q; ++z) buf_store<T>(uc[z] + d[z], ur, off, sbase + splane * z);
  }
}

}  // namespace vps
