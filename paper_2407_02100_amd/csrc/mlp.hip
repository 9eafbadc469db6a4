// Learned per-eigenmode scaling of the patch inverse: features, exact training
// targets, MLP forward/backward/Adam and per-patch inference (FP32 network,
// FP64 targets).
#include <cmath>
#include <mutex>

#include "kernels.h"
#include "mlp_launch.h"

namespace vps {

namespace {

constexpr int H = kMlpHidden;

__device__ inline void patch_vertex(long long j, int ncell, int dim, int* v) {
  const long long m = ncell - 1;
  v[0] = (int)(j % m) + 1;
  v[1] = (int)((j / m) % m) + 1;
  v[2] = (dim == 3) ? (int)(j / (m * m)) + 1 : 1;
}

__device__ inline double patch_cell_rho(const double* rho, int ncell, int dim, const int* v, int c) {
  const int cx = v[0] - 1 + (c & 1), cy = v[1] - 1 + ((c >> 1) & 1);
  const int cz = (dim == 3) ? v[2] - 1 + ((c >> 2) & 1) : 0;
  return rho[(size_t)cx + (size_t)ncell * ((size_t)cy + (size_t)ncell * (size_t)cz)];
}

// x[j][c] = log(rho_c / rhobar_j) over the patch's cells.
__global__ void __launch_bounds__(kBlock) features_kernel(const double* __restrict__ rho, int ncell, int dim,
                                                          long long npatch, float* __restrict__ x) {
  const long long j = blockIdx.x * (long long)kBlock + threadIdx.x;
  if (j >= npatch) return;
  int v[3];
  patch_vertex(j, ncell, dim, v);
  const int nc = 1 << dim;
  double r[8], s = 0.0;
  for (int c = 0; c < nc; ++c) {
    r[c] = patch_cell_rho(rho, ncell, dim, v, c);
    s += r[c];
  }
  const double mean = s / nc;
  for (int c = 0; c < nc; ++c) x[j * nc + c] = (float)log(r[c] / mean);
}

__global__ void __launch_bounds__(kBlock) rho8_kernel(const double* __restrict__ rho, int ncell, int dim,
                                                      long long npatch, double* __restrict__ rho8) {
  const long long j = blockIdx.x * (long long)kBlock + threadIdx.x;
  if (j >= npatch) return;
  int v[3];
  patch_vertex(j, ncell, dim, v);
  const int nc = 1 << dim;
  for (int c = 0; c < nc; ++c) rho8[j * nc + c] = patch_cell_rho(rho, ncell, dim, v, c);
}

__global__ void __launch_bounds__(kBlock) rho8_features_kernel(const double* __restrict__ rho8, long long n, int nc,
                                                               float* __restrict__ x) {
  const long long j = blockIdx.x * (long long)kBlock + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int c = 0; c < nc; ++c) s += rho8[j * nc + c];
  const double mean = s / nc;
  for (int c = 0; c < nc; ++c) x[j * nc + c] = (float)log(rho8[j * nc + c] / mean);
}

// ---- network evaluation, one thread per sample, parameters in LDS ----
struct Net {
  const float* W1;
  const float* b1;
  const float* W2;
  const float* b2;
  const float* W3;
  const float* b3;
};

__device__ inline Net net_view(const float* p, int nin, int nout) {
  Net n;
  n.W1 = p;
  n.b1 = n.W1 + H * nin;
  n.W2 = n.b1 + H;
  n.b2 = n.W2 + H * H;
  n.W3 = n.b2 + H;
  n.b3 = n.W3 + nout * H;
  return n;
}

constexpr int kMaxParams = H * kMlpMaxIn + H + H * H + H + kMlpMaxOut * H + kMlpMaxOut;

__device__ inline void load_params(const float* __restrict__ params, float* sp, int np) {
  for (int i = threadIdx.x; i < np; i += blockDim.x) sp[i] = params[i];
  __syncthreads();
}

__device__ inline void net_eval(const Net& w, int nin, int nout, const float* xin, float* h1, float* h2,
                                float* y) {
  for (int o = 0; o < H; ++o) {
    float a = w.b1[o];
    for (int i = 0; i < nin; ++i) a += w.W1[o * nin + i] * xin[i];
    h1[o] = tanhf(a);
  }
  for (int o = 0; o < H; ++o) {
    float a = w.b2[o];
#pragma unroll 8
    for (int i = 0; i < H; ++i) a += w.W2[o * H + i] * h1[i];
    h2[o] = tanhf(a);
  }
  for (int o = 0; o < nout; ++o) {
    float a = w.b3[o];
#pragma unroll 8
    for (int i = 0; i < H; ++i) a += w.W3[o * H + i] * h2[i];
    y[o] = a;
  }
}

__global__ void __launch_bounds__(kBlock) forward_kernel(const float* __restrict__ params,
                                                         const float* __restrict__ x, long long n, int nin,
                                                         int nout, float* __restrict__ y,
                                                         float* __restrict__ act) {
  __shared__ float sp[kMaxParams];
  load_params(params, sp, mlp_param_count(nin, nout));
  const long long s = blockIdx.x * (long long)kBlock + threadIdx.x;
  if (s >= n) return;
  const Net w = net_view(sp, nin, nout);
  float xin[kMlpMaxIn], h1[H], h2[H], yo[kMlpMaxOut];
  for (int i = 0; i < nin; ++i) xin[i] = x[s * nin + i];
  net_eval(w, nin, nout, xin, h1, h2, yo);
  for (int o = 0; o < nout; ++o) y[s * nout + o] = yo[o];
  if (act) {
    for (int i = 0; i < H; ++i) {
      act[s * 2 * H + i] = h1[i];
      act[s * 2 * H + H + i] = h2[i];
    }
  }
}

// delta[s] = [da2 (H), da1 (H)]
__global__ void __launch_bounds__(kBlock) backward_delta_kernel(const float* __restrict__ params,
                                                                const float* __restrict__ act,
                                                                const float* __restrict__ dy, long long n, int nin,
                                                                int nout, float* __restrict__ delta) {
  __shared__ float sp[kMaxParams];
  load_params(params, sp, mlp_param_count(nin, nout));
  const long long s = blockIdx.x * (long long)kBlock + threadIdx.x;
  if (s >= n) return;
  const Net w = net_view(sp, nin, nout);
  float g[kMlpMaxOut], da2[H];
  for (int o = 0; o < nout; ++o) g[o] = dy[s * nout + o];
  for (int j = 0; j < H; ++j) {
    float a = 0.f;
    for (int o = 0; o < nout; ++o) a += w.W3[o * H + j] * g[o];
    const float h2 = act[s * 2 * H + H + j];
    da2[j] = a * (1.f - h2 * h2);
    delta[s * 2 * H + j] = da2[j];
  }
  for (int i = 0; i < H; ++i) {
    float a = 0.f;
#pragma unroll 8
    for (int j = 0; j < H; ++j) a += w.W2[j * H + i] * da2[j];
    const float h1 = act[s * 2 * H + i];
    delta[s * 2 * H + H + i] = a * (1.f - h1 * h1);
  }
}

// partial[split][p] = sum over the split's samples of the sample's gradient of parameter p
__global__ void __launch_bounds__(kBlock) grad_partial_kernel(const float* __restrict__ x,
                                                              const float* __restrict__ act,
                                                              const float* __restrict__ dy,
                                                              const float* __restrict__ delta, long long n,
                                                              int nin, int nout, long long chunk,
                                                              float* __restrict__ partial) {
  const int np = mlp_param_count(nin, nout);
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= np) return;
  const long long s0 = blockIdx.y * chunk;
  const long long s1 = (s0 + chunk < n) ? s0 + chunk : n;
  // decode the parameter
  const int oW1 = 0, ob1 = oW1 + H * nin, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H, ob3 = oW3 + nout * H;
  float acc = 0.f;
  if (p < ob1) {  // W1[o][i]: da1[o] x[i]
    const int o = (p - oW1) / nin, i = (p - oW1) % nin;
    for (long long s = s0; s < s1; ++s) acc += delta[s * 2 * H + H + o] * x[s * nin + i];
  } else if (p < oW2) {  // b1[o]
    const int o = p - ob1;
    for (long long s = s0; s < s1; ++s) acc += delta[s * 2 * H + H + o];
  } else if (p < ob2) {  // W2[o][i]: da2[o] h1[i]
    const int o = (p - oW2) / H, i = (p - oW2) % H;
    for (long long s = s0; s < s1; ++s) acc += delta[s * 2 * H + o] * act[s * 2 * H + i];
  } else if (p < oW3) {  // b2[o]
    const int o = p - ob2;
    for (long long s = s0; s < s1; ++s) acc += delta[s * 2 * H + o];
  } else if (p < ob3) {  // W3[o][i]: dy[o] h2[i]
    const int o = (p - oW3) / H, i = (p - oW3) % H;
    for (long long s = s0; s < s1; ++s) acc += dy[s * nout + o] * act[s * 2 * H + H + i];
  } else {  // b3[o]
    const int o = p - ob3;
    for (long long s = s0; s < s1; ++s) acc += dy[s * nout + o];
  }
  partial[(size_t)blockIdx.y * np + p] = acc;
}

__global__ void __launch_bounds__(kBlock) grad_final_kernel(const float* __restrict__ partial, int nsplit, int np,
                                                            float* __restrict__ g) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= np) return;
  float a = 0.f;
  for (int k = 0; k < nsplit; ++k) a += partial[(size_t)k * np + p];
  g[p] = a;
}

__device__ inline double block_sum_d(double v, double* red) {
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

__global__ void __launch_bounds__(kBlock) loss_grad_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                           long long total, float scale, float* __restrict__ dy,
                                                           float* __restrict__ partial) {
  __shared__ double red[kBlock];
  double acc = 0.0;
  for (long long e = blockIdx.x * (long long)kBlock + threadIdx.x; e < total; e += (long long)gridDim.x * kBlock) {
    const float d = y[e] - t[e];
    dy[e] = 2.f * scale * d;
    acc += (double)d * (double)d;
  }
  const double s = block_sum_d(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = (float)s;
}

__global__ void __launch_bounds__(kBlock) loss_final_kernel(const float* __restrict__ partial, int nblk, float scale,
                                                            float* __restrict__ loss) {
  __shared__ double red[kBlock];
  double a = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kBlock) a += partial[i];
  const double s = block_sum_d(a, red);
  if (threadIdx.x == 0) *loss = (float)(s * scale);
}

__global__ void __launch_bounds__(kBlock) adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                      float* __restrict__ m, float* __restrict__ v, int np, float lr,
                                                      float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= np) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void __launch_bounds__(kBlock) infer_kernel(const double* __restrict__ rho, int ncell, int dim,
                                                       const float* __restrict__ params, int nin, int nout,
                                                       long long npatch, float* __restrict__ scal,
                                                       int* __restrict__ counter) {
  __shared__ float sp[kMaxParams];
  load_params(params, sp, mlp_param_count(nin, nout));
  const long long j = blockIdx.x * (long long)kBlock + threadIdx.x;
  if (j >= npatch) return;
  const Net w = net_view(sp, nin, nout);
  int v[3];
  patch_vertex(j, ncell, dim, v);
  double r[8], s = 0.0;
  for (int c = 0; c < nin; ++c) {
    r[c] = patch_cell_rho(rho, ncell, dim, v, c);
    s += r[c];
  }
  const double mean = s / nin;
  float xin[kMlpMaxIn], h1[H], h2[H], y[kMlpMaxOut];
  for (int c = 0; c < nin; ++c) xin[c] = (float)log(r[c] / mean);
  net_eval(w, nin, nout, xin, h1, h2, y);
  bool ok = true;
  for (int o = 0; o < nout; ++o) ok = ok && isfinite(y[o]);
  for (int o = 0; o < nout; ++o) {
    float c = 1.f;
    if (ok) c = fminf(fmaxf(expf(y[o]), 0.25f), 4.f);
    scal[j * nout + o] = c;
  }
  if (!ok) atomicAdd(counter, 1);
}

// ---- exact targets of Q2 patches in 3D: one wavefront per patch ----
struct TargetArgs {
  double Mi[2][9];  // interior q x q block of the cell-h half of the patch mass matrix
  double Ki[2][9];
  double T[9];      // eigenvectors, T[i*3+m]
  double lam[3];
};

__global__ void __launch_bounds__(64) targets_kernel(const TargetArgs a, const double* __restrict__ rho8,
                                                     double* __restrict__ cstar, float* __restrict__ logt) {
  constexpr int Q = 3, N = 27;
  __shared__ double A[N * N];
  __shared__ double S[N * N];
  __shared__ double W[N * N];
  __shared__ double r8[8];
  __shared__ double rhs[N];
  __shared__ double sol[N];
  const long long j = blockIdx.x;
  const int lane = threadIdx.x;
  if (lane < 8) r8[lane] = rho8[j * 8 + lane];
  __syncthreads();
  double rbar = 0.0;
  for (int c = 0; c < 8; ++c) rbar += r8[c];
  rbar *= 0.125;
  // A_j(rho) on the interior nodes: sum over cells of rho_c times the cell's Kronecker sum
  for (int e = lane; e < N * N; e += 64) {
    const int o = e / N, i = e % N;
    const int ox = o % Q, oy = (o / Q) % Q, oz = o / (Q * Q);
    const int ix = i % Q, iy = (i / Q) % Q, iz = i / (Q * Q);
    double v = 0.0;
    for (int c = 0; c < 8; ++c) {
      const int hx = c & 1, hy = (c >> 1) & 1, hz = (c >> 2) & 1;
      const double mx = a.Mi[hx][ox * Q + ix], my = a.Mi[hy][oy * Q + iy], mz = a.Mi[hz][oz * Q + iz];
      const double kx = a.Ki[hx][ox * Q + ix], ky = a.Ki[hy][oy * Q + iy], kz = a.Ki[hz][oz * Q + iz];
      v += r8[c] * (kx * my * mz + mx * ky * mz + mx * my * kz);
    }
    A[e] = v;
    // S[i][m] = T[ix][mx] T[iy][my] T[iz][mz]  (row = node o, column = mode i here)
    S[e] = a.T[ox * Q + ix] * a.T[oy * Q + iy] * a.T[oz * Q + iz];
  }
  __syncthreads();
  for (int e = lane; e < N * N; e += 64) {  // W = A S
    const int r = e / N, m = e % N;
    double s = 0.0;
    for (int l = 0; l < N; ++l) s += A[r * N + l] * S[l * N + m];
    W[e] = s;
  }
  __syncthreads();
  for (int e = lane; e < N * N; e += 64) {  // Y = S^T W  (into A)
    const int m = e / N, mp = e % N;
    double s = 0.0;
    for (int l = 0; l < N; ++l) s += S[l * N + m] * W[l * N + mp];
    A[e] = s;
  }
  __syncthreads();
  for (int e = lane; e < N * N; e += 64) W[e] = A[e] * A[e];  // Y o Y
  if (lane < N) rhs[lane] = A[lane * N + lane];
  __syncthreads();
  // Cholesky W = L L^T (lower triangle of W)
  for (int k = 0; k < N; ++k) {
    if (lane == 0) {
      double d = W[k * N + k];
      for (int p = 0; p < k; ++p) d -= W[k * N + p] * W[k * N + p];
      W[k * N + k] = sqrt(d);
    }
    __syncthreads();
    const int i = k + 1 + lane;
    if (i < N) {
      double s = W[i * N + k];
      for (int p = 0; p < k; ++p) s -= W[i * N + p] * W[k * N + p];
      W[i * N + k] = s / W[k * N + k];
    }
    __syncthreads();
  }
  if (lane == 0) {
    for (int i = 0; i < N; ++i) {  // L z = rhs
      double s = rhs[i];
      for (int p = 0; p < i; ++p) s -= W[i * N + p] * sol[p];
      sol[i] = s / W[i * N + i];
    }
    for (int i = N - 1; i >= 0; --i) {  // L^T d = z
      double s = sol[i];
      for (int p = i + 1; p < N; ++p) s -= W[p * N + i] * sol[p];
      sol[i] = s / W[i * N + i];
    }
  }
  __syncthreads();
  if (lane < N) {
    const int mx = lane % Q, my = (lane / Q) % Q, mz = lane / (Q * Q);
    const double c = rbar * (a.lam[mx] + a.lam[my] + a.lam[mz]) * sol[lane];
    cstar[j * N + lane] = c;
    if (logt) logt[j * N + lane] = (float)log(fmin(fmax(c, 0.25), 4.0));
  }
}

// Exact dense local solver of a Q2 patch (3D): B_j = A_j(rho)^{-1}, A_j the
// interior block of the sum over the patch's 8 cells of rho_c times the cell's
// Kronecker sum (eq:main:2 with the exact inverse).  One wave per patch:
// assemble A_j in LDS, Cholesky A_j = L L^T (lane 0 the pivots, the column in
// parallel), then lane i < 27 solves L L^T x = e_i for column i of B_j.
// binv: npatch x 27 x 27 FP64, patch-major (B_j symmetric, so either index
// order).
struct ExactArgs {
  double Mi[2][9];  // interior 3 x 3 block of the cell-h half of the level's 1D patch mass matrix
  double Ki[2][9];
};

__global__ void __launch_bounds__(64) exact_inverse_kernel(const ExactArgs a, const double* __restrict__ rho, int ncell,
                                                           double* __restrict__ binv) {
  constexpr int Q = 3, N = 27;
  __shared__ double A[N * N];
  __shared__ double r8[8];
  const long long j = blockIdx.x;
  const int lane = threadIdx.x;
  if (lane < 8) {
    int v[3];
    patch_vertex(j, ncell, 3, v);
    r8[lane] = patch_cell_rho(rho, ncell, 3, v, lane);
  }
  __syncthreads();
  for (int e = lane; e < N * N; e += 64) {
    const int o = e / N, i = e % N;
    const int ox = o % Q, oy = (o / Q) % Q, oz = o / (Q * Q);
    const int ix = i % Q, iy = (i / Q) % Q, iz = i / (Q * Q);
    double v = 0.0;
    for (int c = 0; c < 8; ++c) {
      const int hx = c & 1, hy = (c >> 1) & 1, hz = (c >> 2) & 1;
      const double mx = a.Mi[hx][ox * Q + ix], my = a.Mi[hy][oy * Q + iy], mz = a.Mi[hz][oz * Q + iz];
      const double kx = a.Ki[hx][ox * Q + ix], ky = a.Ki[hy][oy * Q + iy], kz = a.Ki[hz][oz * Q + iz];
      v += r8[c] * (kx * my * mz + mx * ky * mz + mx * my * kz);
    }
    A[e] = v;
  }
  __syncthreads();
  for (int k = 0; k < N; ++k) {  // lower triangle of A <- L
    if (lane == 0) {
      double d = A[k * N + k];
      for (int p = 0; p < k; ++p) d -= A[k * N + p] * A[k * N + p];
      A[k * N + k] = sqrt(d);
    }
    __syncthreads();
    const int i = k + 1 + lane;
    if (i < N) {
      double s = A[i * N + k];
      for (int p = 0; p < k; ++p) s -= A[i * N + p] * A[k * N + p];
      A[i * N + k] = s / A[k * N + k];
    }
    __syncthreads();
  }
  if (lane < N) {
    double x[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {  // L y = e_lane
      double s = (i == lane) ? 1.0 : 0.0;
#pragma unroll
      for (int p = 0; p < i; ++p) s -= A[i * N + p] * x[p];
      x[i] = s / A[i * N + i];
    }
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {  // L^T x = y
      double s = x[i];
#pragma unroll
      for (int p = i + 1; p < N; ++p) s -= A[p * N + i] * x[p];
      x[i] = s / A[i * N + i];
    }
    double* out = binv + j * (N * N) + lane;
#pragma unroll
    for (int i = 0; i < N; ++i) out[i * N] = x[i];  // column lane of B_j: B[i][lane]
  }
}

// One color step of the exact local solver: u_I += B_j r_I for every patch of
// the color (r = b - A u of the current iterate, computed before the step; the
// color's patches do not read each other's writes).  One wave per patch.
__global__ void __launch_bounds__(64) exact_apply_kernel(double* __restrict__ u, const double* __restrict__ r,
                                                         const double* __restrict__ binv, int n1, int ncell, int v0x,
                                                         int v0y, int v0z, int npx, int npy, long long ncolor) {
  constexpr int Q = 3, N = 27;
  __shared__ double rs[N];
  const long long t = blockIdx.x;
  if (t >= ncolor) return;
  const int lane = threadIdx.x;
  const int px = (int)(t % npx), py = (int)((t / npx) % npy), pz = (int)(t / ((long long)npx * npy));
  const int vx = v0x + 2 * px, vy = v0y + 2 * py, vz = v0z + 2 * pz;
  const long long m = ncell - 1;
  const long long j = (long long)(vx - 1) + m * ((long long)(vy - 1) + m * (long long)(vz - 1));
  size_t node = 0;
  if (lane < N) {
    const int ix = lane % Q, iy = (lane / Q) % Q, iz = lane / (Q * Q);
    node = (size_t)(2 * (vx - 1) + 1 + ix) + (size_t)n1 * ((size_t)(2 * (vy - 1) + 1 + iy) +
                                                         (size_t)n1 * (size_t)(2 * (vz - 1) + 1 + iz));
    rs[lane] = r[node];
  }
  __syncthreads();
  if (lane < N) {
    const double* B = binv + j * (N * N);
    double d = 0.0;
#pragma unroll
    for (int q = 0; q < N; ++q) d += B[q * N + lane] * rs[q];
    u[node] += d;
  }
}

inline unsigned blocks_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Grow a work buffer; waits for the stream first so that no queued kernel
// still uses the old allocation when it is freed.
hipError_t grow(float** buf, size_t* cap, size_t need, hipStream_t s) {
  if (*cap >= need) return hipSuccess;
  hipError_t e0 = hipStreamSynchronize(s);
  if (e0 != hipSuccess) return e0;
  if (*buf) (void)hipFree(*buf);
  *buf = nullptr;
  *cap = 0;
  hipError_t e = hipMalloc(buf, need * sizeof(float));
  if (e == hipSuccess) *cap = need;
  return e;
}

}  // namespace

hipError_t mlp_ensure(MlpWork* w) {
  if (!w->counter) {
    hipError_t e = hipMalloc(&w->counter, sizeof(int));
    if (e != hipSuccess) return e;
  }
  if (!w->hcounter) {
    hipError_t e = hipHostMalloc(&w->hcounter, sizeof(int), 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void mlp_free(MlpWork* w) {
  if (w->delta) (void)hipFree(w->delta);
  if (w->partial) (void)hipFree(w->partial);
  if (w->counter) (void)hipFree(w->counter);
  if (w->hcounter) (void)hipHostFree(w->hcounter);
  *w = MlpWork();
}

hipError_t launch_patch_features(const double* rho, int ncell, int dim, float* x, hipStream_t s) {
  long long np = 1;
  for (int e = 0; e < dim; ++e) np *= (ncell - 1);
  if (np <= 0) return hipSuccess;
  features_kernel<<<blocks_for(np), kBlock, 0, s>>>(rho, ncell, dim, np, x);
  return hipGetLastError();
}

hipError_t launch_patch_rho8(const double* rho, int ncell, int dim, double* rho8, hipStream_t s) {
  long long np = 1;
  for (int e = 0; e < dim; ++e) np *= (ncell - 1);
  if (np <= 0) return hipSuccess;
  rho8_kernel<<<blocks_for(np), kBlock, 0, s>>>(rho, ncell, dim, np, rho8);
  return hipGetLastError();
}

hipError_t launch_rho8_features(const double* rho8, long long n, int dim, float* x, hipStream_t s) {
  rho8_features_kernel<<<blocks_for(n), kBlock, 0, s>>>(rho8, n, 1 << dim, x);
  return hipGetLastError();
}

hipError_t launch_patch_targets(const double* rho8, long long n, const std::vector<double>* Mh,
                                const std::vector<double>* Kh, const double* T1, const double* lam, double* cstar,
                                float* log_target, hipStream_t s) {
  constexpr int Q = 3, P = 5;
  TargetArgs a;
  for (int h = 0; h < 2; ++h)
    for (int o = 0; o < Q; ++o)
      for (int i = 0; i < Q; ++i) {
        a.Mi[h][o * Q + i] = Mh[h][o * P + i + 1];
        a.Ki[h][o * Q + i] = Kh[h][o * P + i + 1];
      }
  for (int i = 0; i < Q * Q; ++i) a.T[i] = T1[i];
  for (int i = 0; i < Q; ++i) a.lam[i] = lam[i];
  for (long long first = 0; first < n; first += 1 << 30) {
    const long long cnt = (n - first < (1LL << 30)) ? n - first : (1LL << 30);
    targets_kernel<<<(unsigned)cnt, 64, 0, s>>>(a, rho8 + first * 8, cstar + first * 27,
                                                 log_target ? log_target + first * 27 : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_exact_inverses(const double* rho, int ncell, const std::vector<double>* Mh,
                                 const std::vector<double>* Kh, double* binv, hipStream_t s) {
  constexpr int Q = 3, P = 5;
  ExactArgs a;
  for (int h = 0; h < 2; ++h)
    for (int o = 0; o < Q; ++o)
      for (int i = 0; i < Q; ++i) {
        a.Mi[h][o * Q + i] = Mh[h][o * P + i + 1];
        a.Ki[h][o * Q + i] = Kh[h][o * P + i + 1];
      }
  const long long np = (long long)(ncell - 1) * (ncell - 1) * (ncell - 1);
  if (np <= 0) return hipSuccess;
  if (np >= (1LL << 31)) return hipErrorInvalidValue;
  exact_inverse_kernel<<<(unsigned)np, 64, 0, s>>>(a, rho, ncell, binv);
  return hipGetLastError();
}

hipError_t launch_exact_apply(double* u, const double* r, const double* binv, int n1, int ncell, int color,
                              hipStream_t s) {
  int v0[3], np[3];
  for (int e = 0; e < 3; ++e) {
    v0[e] = ((color >> e) & 1) ? 1 : 2;
    np[e] = (v0[e] <= ncell - 1) ? (ncell - 1 - v0[e]) / 2 + 1 : 0;
    if (np[e] == 0) return hipSuccess;
  }
  const long long nc = (long long)np[0] * np[1] * np[2];
  if (nc >= (1LL << 31)) return hipErrorInvalidValue;
  exact_apply_kernel<<<(unsigned)nc, 64, 0, s>>>(u, r, binv, n1, ncell, v0[0], v0[1], v0[2], np[0], np[1], nc);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* params, const float* x, long long n, int nin, int nout, float* y,
                              float* act, hipStream_t s) {
  if (nin > kMlpMaxIn || nout > kMlpMaxOut) return hipErrorInvalidValue;
  if (n == 0) return hipSuccess;
  forward_kernel<<<blocks_for(n), kBlock, 0, s>>>(params, x, n, nin, nout, y, act);
  return hipGetLastError();
}

hipError_t launch_mlp_loss_grad(const float* y, const float* t, long long n, int nout, float* dy, float* loss,
                                MlpWork* w, hipStream_t s) {
  const long long total = n * nout;
  long long g = blocks_for(total);
  if (g > 1024) g = 1024;
  hipError_t e = grow(&w->partial, &w->partial_cap, (size_t)g, s);
  if (e != hipSuccess) return e;
  const float scale = (float)(1.0 / (double)total);
  loss_grad_kernel<<<(unsigned)g, kBlock, 0, s>>>(y, t, total, scale, dy, w->partial);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (loss) {
    loss_final_kernel<<<1, kBlock, 0, s>>>(w->partial, (int)g, scale, loss);
    e = hipGetLastError();
  }
  return e;
}

namespace {

// split of the samples for the partial gradients: at most 64 splits of >= 256 samples
long long backward_splits(long long n) {
  long long nsplit = (n + 255) / 256;
  return nsplit > 64 ? 64 : nsplit;
}

// the three backward kernels on caller-provided work memory: delta (n x 2H floats) and
// partial (splits x parameter count floats), both fully overwritten before they are read
hipError_t backward_kernels(const float* params, const float* x, const float* act, const float* dy, long long n,
                            int nin, int nout, float* dparams, float* delta, float* partial, hipStream_t s) {
  const int np = mlp_param_count(nin, nout);
  const long long nsplit = backward_splits(n);
  const long long chunk = (n + nsplit - 1) / nsplit;
  backward_delta_kernel<<<blocks_for(n), kBlock, 0, s>>>(params, act, dy, n, nin, nout, delta);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 grid((np + kBlock - 1) / kBlock, (unsigned)nsplit);
  grad_partial_kernel<<<grid, kBlock, 0, s>>>(x, act, dy, delta, n, nin, nout, chunk, partial);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  grad_final_kernel<<<(np + kBlock - 1) / kBlock, kBlock, 0, s>>>(partial, (int)nsplit, np, dparams);
  return hipGetLastError();
}

// Work memory of the allocation-free backward (vps_mlp_backward_noalloc): one
// copy per GPU for the life of the process, shared by every call on that GPU.
// Host code reaches it only through the address hipGetSymbolAddress returns
// for the current device (g_scratch_dev), never through the array's name.
constexpr size_t kScratchFloats = size_t(1) << 20;  // 4 MiB
static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxDevices] = {};

}  // namespace

hipError_t launch_mlp_backward(const float* params, const float* x, const float* act, const float* dy, long long n,
                               int nin, int nout, float* dparams, MlpWork* w, hipStream_t s) {
  if (nin > kMlpMaxIn || nout > kMlpMaxOut) return hipErrorInvalidValue;
  hipError_t e = grow(&w->delta, &w->delta_cap, (size_t)n * 2 * H, s);
  if (e != hipSuccess) return e;
  const int np = mlp_param_count(nin, nout);
  if ((e = grow(&w->partial, &w->partial_cap, (size_t)backward_splits(n) * np, s)) != hipSuccess) return e;
  return backward_kernels(params, x, act, dy, n, nin, nout, dparams, w->delta, w->partial, s);
}

long long mlp_noalloc_max_samples(int nin, int nout) {
  const long long np = mlp_param_count(nin, nout);
  const long long room = (long long)kScratchFloats - 64 * np;  // partials of the largest split count
  return room > 0 ? room / (2 * H) : 0;
}

hipError_t mlp_scratch_setup() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev]) return hipSuccess;
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_dev[dev] = static_cast<float*>(ptr);
  return hipSuccess;
}

hipError_t launch_mlp_backward_noalloc(const float* params, const float* x, const float* act, const float* dy,
                                       long long n, int nin, int nout, float* dparams, hipStream_t s) {
  if (nin > kMlpMaxIn || nout > kMlpMaxOut) return hipErrorInvalidValue;
  if (n <= 0 || n > mlp_noalloc_max_samples(nin, nout)) return hipErrorInvalidValue;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  float* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev >= 0 && dev < kMaxDevices) base = g_scratch_dev[dev];
  }
  if (!base) return hipErrorNotInitialized;  // mlp_scratch_setup has not run on this device
  const size_t np = (size_t)mlp_param_count(nin, nout);
  float* partial = base;                                       // 64 x np floats at most
  float* delta = base + 64 * np;                               // n x 2H floats
  return backward_kernels(params, x, act, dy, n, nin, nout, dparams, delta, partial, s);
}

hipError_t launch_mlp_adam(float* params, const float* g, float* m, float* v, int np, int step, float lr, float b1,
                           float b2, float eps, hipStream_t s) {
  const float c1 = (float)(1.0 - std::pow((double)b1, step));
  const float c2 = (float)(1.0 - std::pow((double)b2, step));
  adam_kernel<<<(np + kBlock - 1) / kBlock, kBlock, 0, s>>>(params, g, m, v, np, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t mlp_infer_patches(const double* rho, int ncell, int dim, const float* params, int nin, int nout,
                             long long npatch, float* scal, long long* fallback, MlpWork* w, hipStream_t s) {
  if (nin > kMlpMaxIn || nout > kMlpMaxOut) return hipErrorInvalidValue;
  hipError_t e = hipMemsetAsync(w->counter, 0, sizeof(int), s);
  if (e != hipSuccess) return e;
  infer_kernel<<<blocks_for(npatch), kBlock, 0, s>>>(rho, ncell, dim, params, nin, nout, npatch, scal, w->counter);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(w->hcounter, w->counter, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  *fallback = *w->hcounter;
  return hipSuccess;
}

}  // namespace vps
