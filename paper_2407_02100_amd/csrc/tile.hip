// Launchers of the tile kernels (operator, restriction, prolongation), the
// variable-coefficient operator and the patch-shape helpers.
#include "kernels.h"
#include "launch.h"

namespace vps {

namespace {

template <typename T, int KIND, int K, int D, int TC>
hipError_t go_tile(const TileLaunch& L, hipStream_t s) {
  using Sh = TileShape<KIND, K, TC>;
  using KS = TileKernelShape<T, KIND, K, D, TC>;
  if constexpr ((KS::BUF0 + KS::BUF1) * sizeof(T) > 65536) {
    return hipErrorInvalidValue;  // this tile does not fit the workgroup LDS (3D, k = 5: streaming kernels only)
  } else {
  static_assert(sizeof(TileArgs<T, KIND, K, TC>) <= 4096, "kernel arguments exceed 4 KiB");
  TileArgs<T, KIND, K, TC> a;
  a.in = (const T*)L.in;
  a.b = (const T*)L.b;
  a.out = (T*)L.out;
  a.n1_in = L.n1_in;
  a.n1_out = L.n1_out;
  for (int i = 0; i < Sh::NO * Sh::NI; ++i) a.G0[i] = (T)L.G0[i];
  if (KIND == TILE_OPERATOR)
    for (int i = 0; i < Sh::NO * Sh::NI; ++i) a.G1[i] = (T)L.G1[i];
  dim3 grid(L.tiles, L.tiles, D == 3 ? L.tiles : 1);
  tile_kernel<T, KIND, K, D, TC><<<grid, kBlock, 0, s>>>(a);
  return hipGetLastError();
  }
}

template <typename T, int K, int D>
struct VarOpArgs {
  const T* __restrict__ u;
  const T* __restrict__ b;
  T* __restrict__ out;
  const T* __restrict__ rho;
  int n1, ncell;
  T Mc[(K + 1) * (K + 1)];
  T Kc[(K + 1) * (K + 1)];
};

// (A u)_g = sum over the cells c containing node g of rho_c (A^c u_c)_g, with
// A^c the Kronecker sum of the 1D cell matrices.  One thread per node.
template <typename T, int K, int D>
__global__ void __launch_bounds__(kBlock) op_var_kernel(const VarOpArgs<T, K, D> a) {
  const int n1 = a.n1;
  const size_t total = (D == 3) ? (size_t)n1 * n1 * n1 : (size_t)n1 * n1;
  for (size_t g = blockIdx.x * (size_t)kBlock + threadIdx.x; g < total; g += (size_t)gridDim.x * kBlock) {
    int idx[3] = {(int)(g % n1), (int)((g / n1) % n1), (D == 3) ? (int)(g / ((size_t)n1 * n1)) : 0};
    bool dir = false;
    for (int e = 0; e < D; ++e) dir = dir || idx[e] == 0 || idx[e] == n1 - 1;
    if (dir) {
      a.out[g] = T(0);
      continue;
    }
    // candidate cells per direction: (cell, local index)
    int cc[3][2], ll[3][2], nc[3];
    for (int e = 0; e < 3; ++e) {
      if (e >= D) { cc[e][0] = 0; ll[e][0] = 0; nc[e] = 1; continue; }
      const int i = idx[e];
      if (i % K == 0) {
        cc[e][0] = i / K - 1; ll[e][0] = K;
        cc[e][1] = i / K;     ll[e][1] = 0;
        nc[e] = 2;
      } else {
        cc[e][0] = i / K; ll[e][0] = i % K; nc[e] = 1;
      }
    }
    T acc = T(0);
    for (int jz = 0; jz < nc[2]; ++jz)
      for (int jy = 0; jy < nc[1]; ++jy)
        for (int jx = 0; jx < nc[0]; ++jx) {
          const int cx = cc[0][jx], cy = cc[1][jy], cz = cc[2][jz];
          const int ax = ll[0][jx], ay = ll[1][jy], az = ll[2][jz];
          const T r = a.rho[(size_t)cx + (size_t)a.ncell * ((size_t)cy + (size_t)a.ncell * (size_t)cz)];
          T s = T(0);
          const int zcnt = (D == 3) ? K + 1 : 1;
          for (int lz = 0; lz < zcnt; ++lz) {
            const T mz = (D == 3) ? a.Mc[az * (K + 1) + lz] : T(1);
            const T kz = (D == 3) ? a.Kc[az * (K + 1) + lz] : T(0);
            for (int ly = 0; ly <= K; ++ly) {
              const T my = a.Mc[ay * (K + 1) + ly];
              const T ky = a.Kc[ay * (K + 1) + ly];
              const size_t row = (size_t)(cx * K) +
                                 (size_t)n1 * ((size_t)(cy * K + ly) + (size_t)n1 * (size_t)(D == 3 ? cz * K + lz : 0));
              T sm = T(0), sk = T(0);
#pragma unroll
              for (int lx = 0; lx <= K; ++lx) {
                const T uv = a.u[row + lx];
                sm += a.Mc[ax * (K + 1) + lx] * uv;
                sk += a.Kc[ax * (K + 1) + lx] * uv;
              }
              s += sk * my * mz + sm * (ky * mz + my * kz);
            }
          }
          acc += r * s;
        }
    a.out[g] = (a.b != nullptr) ? a.b[g] - acc : acc;
  }
}

}  // namespace

template <typename T, int K, int D>
hipError_t launch_operator(const TileLaunch& L, hipStream_t s) {
  return go_tile<T, TILE_OPERATOR, K, D, op_tc(K, D)>(L, s);
}
template <typename T, int K, int D>
hipError_t launch_restrict(const TileLaunch& L, hipStream_t s) {
  return go_tile<T, TILE_RESTRICT, K, D, restrict_tc(K, D)>(L, s);
}
template <typename T, int K, int D>
hipError_t launch_prolong(const TileLaunch& L, hipStream_t s) {
  return go_tile<T, TILE_PROLONG, K, D, prolong_tc(K, D)>(L, s);
}

template <typename T, int K, int D>
hipError_t launch_operator_var(const VarOpLaunch& L, hipStream_t s) {
  static_assert(sizeof(VarOpArgs<T, K, D>) <= 4096, "kernel arguments exceed 4 KiB");
  VarOpArgs<T, K, D> a;
  a.u = (const T*)L.u;
  a.b = (const T*)L.b;
  a.out = (T*)L.out;
  a.rho = (const T*)L.rho;
  a.n1 = L.n1;
  a.ncell = L.ncell;
  for (int i = 0; i < (K + 1) * (K + 1); ++i) {
    a.Mc[i] = (T)L.Mc[i];
    a.Kc[i] = (T)L.Kc[i];
  }
  const size_t total = (D == 3) ? (size_t)L.n1 * L.n1 * L.n1 : (size_t)L.n1 * L.n1;
  size_t g = (total + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  op_var_kernel<T, K, D><<<(unsigned)g, kBlock, 0, s>>>(a);
  return hipGetLastError();
}

#define VPS_TILE_INST(T, K, D)                                                   \
  template hipError_t launch_operator<T, K, D>(const TileLaunch&, hipStream_t);  \
  template hipError_t launch_restrict<T, K, D>(const TileLaunch&, hipStream_t);  \
  template hipError_t launch_prolong<T, K, D>(const TileLaunch&, hipStream_t);   \
  template hipError_t launch_operator_var<T, K, D>(const VarOpLaunch&, hipStream_t);
#define VPS_TILE_INST_K(K) \
  VPS_TILE_INST(double, K, 2) VPS_TILE_INST(double, K, 3) VPS_TILE_INST(float, K, 2) VPS_TILE_INST(float, K, 3)
VPS_TILE_INST_K(1)
VPS_TILE_INST_K(2)
VPS_TILE_INST_K(3)
VPS_TILE_INST_K(4)
VPS_TILE_INST_K(5)

// ---- patch shape helpers ----
template <typename T, int K, int D, int COEF>
static int lds_of(int pb) {
  switch (pb) {
    case 1: return PatchKernelShape<T, K, D, COEF, 1>::LDS_BYTES;
    case 2: return PatchKernelShape<T, K, D, COEF, 2>::LDS_BYTES;
    case 4: return PatchKernelShape<T, K, D, COEF, 4>::LDS_BYTES;
  }
  return 1 << 30;
}

template <typename T, int K, int D>
static int lds_coef(int coef, int pb) {
  if (coef == 0) return lds_of<T, K, D, 0>(pb);
  if (coef == 1) return lds_of<T, K, D, 1>(pb);
  return lds_of<T, K, D, 2>(pb);
}

static int patch_lds_bytes(int K, int D, int coef, int pb, bool fp64) {
#define VPS_LDS_CASE(KK, DD)                                                                  \
  if (K == KK && D == DD) return fp64 ? lds_coef<double, KK, DD>(coef, pb) : lds_coef<float, KK, DD>(coef, pb);
  VPS_LDS_CASE(1, 2) VPS_LDS_CASE(1, 3) VPS_LDS_CASE(2, 2) VPS_LDS_CASE(2, 3)
  VPS_LDS_CASE(3, 2) VPS_LDS_CASE(3, 3) VPS_LDS_CASE(4, 2) VPS_LDS_CASE(4, 3) VPS_LDS_CASE(5, 2) VPS_LDS_CASE(5, 3)
#undef VPS_LDS_CASE
  return 1 << 30;
}

bool valid_patches_per_block(int pb) { return pb == 1 || pb == 2 || pb == 4; }

bool patches_per_block_fits(int K, int D, int coef, int pb, bool fp64) {
  return patch_lds_bytes(K, D, coef, pb, fp64) + 4096 <= 65536;
}

int default_patches_per_block(int K, int D, int coef, bool fp64) {
  // the largest batch whose LDS stays below 40 KiB (room for 3+ workgroups per CU)
  for (int pb : {4, 2, 1})
    if (patch_lds_bytes(K, D, coef, pb, fp64) <= 40 * 1024) return pb;
  for (int pb : {2, 1})
    if (patch_lds_bytes(K, D, coef, pb, fp64) + 4096 <= 65536) return pb;
  return 1;
}

}  // namespace vps
