// Host-side launchers of libvps kernels (library-internal).
//
// Each launcher takes runtime descriptions (device pointers, sizes, and the
// level's 1D matrices as host FP64 arrays), builds the kernel's argument
// struct in the kernel's arithmetic type and launches on the given stream.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace vps {

// Tile sizes (cells per direction) of the operator and transfer kernels.
constexpr int op_tc(int K, int D) { return D == 2 ? (K <= 2 ? 4 : 2) : (K == 1 ? 8 : (K == 2 ? 4 : (K <= 4 ? 2 : 1))); }
constexpr int restrict_tc(int K, int D) { return D == 2 ? 2 : (K <= 2 ? 2 : 1); }
constexpr int prolong_tc(int K, int D) { return D == 2 ? 2 : (K <= 2 ? 2 : 1); }

// Patches per workgroup along x that the automatic choice uses.
int default_patches_per_block(int K, int D, int coef, bool fp64);
// Supported explicit choices.
bool valid_patches_per_block(int pb);
// Whether the LDS-staged kernel with that batch fits the workgroup LDS.
bool patches_per_block_fits(int K, int D, int coef, int pb, bool fp64);

struct PatchLaunch {
  void* u;
  const void* b;
  const void* rho;     // per-cell coefficient of the level (same dtype as u), coef != 0
  const float* scal;   // per-patch eigenmode factors, coef == 2
  int n1, ncell;
  int color;           // bit e = parity of the vertex index along direction e
  int coef;            // 0, 1, 2
  int pb;              // patches per workgroup along x
  const double* M[2];  // Q x P each (see PatchMats)
  const double* Kst[2];
  const double* T1;    // Q x Q
  const double* lam;   // Q
  // one-patch-per-wavefront kernel (3D, rho = 1): even/odd blocks of T and the
  // reciprocal eigenvalue sums in the internal mode order (device, dtype of u)
  const double* Te;    // K x K
  const double* To;    // (K-1) x (K-1)
  const double* lam_int;  // Q eigenvalues in the even/odd mode order (host), or null
  int order;              // vps_config.patch_order (3D one-patch-per-wave kernel)
  int ppw;                // 3D, rho = 1, K = 2..4: patches per wavefront (1 or 2)
  int row2;               // 2D, rho = 1, K = 2..5: row of patches per wave (0 automatic, 1 always, 2 never)
  int vlo, vhi;           // vertex range (inclusive) in the slowest direction; vhi = 0: all vertices
};

template <typename T, int K, int D>
hipError_t launch_patch_color(const PatchLaunch& L, hipStream_t s);
// Separated smoother (3D, constant coefficient): u_int += A_j^{-1} r_int on the patches of L.color.
template <typename T, int K>
hipError_t launch_patch_solve(const PatchLaunch& L, const void* r, hipStream_t s);

struct TileLaunch {
  const void* in;
  const void* b;   // operator only: r = b - A u when non-null
  void* out;
  int n1_in, n1_out;
  int tiles;       // tiles per direction
  const double* G0;  // NO x NI
  const double* G1;  // NO x NI (operator stiffness) or null
};

// Row-streaming 2D operator / residual (constant coefficient).
struct Stream2Launch {
  const void* in;
  const void* b;   // r = b - A u when non-null
  void* out;
  int n1, ncell;
  const double* Mc;  // (K+1) x (K+1) cell mass matrix (h-scaled)
  const double* Kc;  // ... and stiffness matrix
};
template <typename T, int K>
hipError_t launch_stream2_operator(const Stream2Launch& L, hipStream_t s);
// 2D transfers on the same struct: ncell = coarse cells; restriction: Mc = the
// restriction rows (K x (4K+1)), Kc = the coarse-cell block ((K+1) x (2K+1));
// prolongation: Mc = the fine rows of one coarse cell (2K x (K+1)).
template <typename T, int K>
hipError_t launch_stream2_restrict(const Stream2Launch& L, hipStream_t s);
template <typename T, int K>
hipError_t launch_stream2_prolong(const Stream2Launch& L, hipStream_t s);

// Plane-streaming 3D kernels (constant coefficient): operator / residual and restriction.
struct StreamLaunch {
  const void* in;
  const void* b;      // operator only: out = b - A u when non-null
  void* out;
  int n1_in, n1_out;
  int ncell_out;      // cells per direction of the output grid; prolongation: of the coarse input grid
  const double* G0;   // PO x W period rows (operator mass / restriction / prolongation)
  const double* G1;   // PO x W operator stiffness period rows, or null
  const double* Z0;   // ZO x (ZIN+1) z cell table (operator mass / restriction / prolongation)
  const double* Z1;   // ZO x (ZIN+1) operator cell stiffness, or null
};
template <typename T, int K>
hipError_t launch_stream_operator(const StreamLaunch& L, hipStream_t s);
template <typename T, int K>
hipError_t launch_stream_restrict(const StreamLaunch& L, hipStream_t s);
template <typename T, int K>
hipError_t launch_stream_prolong(const StreamLaunch& L, hipStream_t s);

template <typename T, int K, int D>
hipError_t launch_operator(const TileLaunch& L, hipStream_t s);
template <typename T, int K, int D>
hipError_t launch_restrict(const TileLaunch& L, hipStream_t s);
template <typename T, int K, int D>
hipError_t launch_prolong(const TileLaunch& L, hipStream_t s);

// Variable-coefficient operator (one thread per node, sum over the node's cells).
struct VarOpLaunch {
  const void* u;
  const void* b;
  void* out;
  const void* rho;
  int n1, ncell;
  const double* Mc;  // (K+1)^2 cell mass  (h-scaled)
  const double* Kc;  // (K+1)^2 cell stiffness (h-scaled)
};
template <typename T, int K, int D>
hipError_t launch_operator_var(const VarOpLaunch& L, hipStream_t s);

// Coarse solvers.
struct CoarseFdmLaunch {
  const void* b;
  void* x;
  int n0;           // free nodes per direction
  const void* T0;   // n0 x n0, device, in the kernel's type
  const void* lam0; // n0, device, in the kernel's type
};
template <typename T, int D>
hipError_t launch_coarse_fdm(const CoarseFdmLaunch& L, hipStream_t s);
constexpr int coarse_fdm_max_n0(int D) { return D == 3 ? 15 : 63; }

template <typename T>
hipError_t launch_coarse_dense(const void* Ainv, const int* free_idx, int nfree, const void* b, void* x,
                               size_t nodes, hipStream_t s);

// Vector kernels.
template <typename T>
hipError_t launch_fill(void* x, double v, size_t n, hipStream_t s);
template <typename Ti, typename To>
hipError_t launch_cast(const void* in, void* out, size_t n, hipStream_t s);
template <typename T>
hipError_t launch_axpy(double a, const void* x, void* y, size_t n, hipStream_t s);  // y += a x
hipError_t launch_xpay(const double* x, double a, double* y, size_t n, hipStream_t s);  // y = x + a y
// x += alpha p (x = alpha p if x_zero); r = r_in - alpha q (r_in may be r); r32 = (float) r if r32 is
// non-null; partial sums of r.r into partial[0..nblk)
hipError_t launch_cg_update(double alpha, const double* p, const double* q, double* x, const double* r_in,
                            double* r, float* r32, bool x_zero, size_t n, double* partial, int* nblk,
                            hipStream_t s);
// partial sums of (r.z) into partial[0..nblk) and, if q is non-null, (z.q) into partial[nblk..2 nblk); z FP32
hipError_t launch_dot_z32(const double* r, const float* z, const double* q, size_t n, double* partial, int* nblk,
                          hipStream_t s);
// p = z + beta p with z FP32
hipError_t launch_xpay_z32(const float* z, double beta, double* p, size_t n, hipStream_t s);
// partial sums of (x.y) into partial[0..nblk) and, if x2/y2 are given, (x2.y2) into partial[nblk..2 nblk)
hipError_t launch_dot_partial(const double* x, const double* y, const double* x2, const double* y2, size_t n,
                              double* partial, int* nblk, hipStream_t s);
// out[j] = sum of partial[j*nblk .. (j+1)*nblk), j < ndot
hipError_t launch_dot_final(const double* partial, int nblk, int ndot, double* out, hipStream_t s);
constexpr int kDotBlocks = 1024;

// Per-cell coefficient of the next coarser level: mean of the 2^D children.
hipError_t launch_coarsen_rho(const double* fine, double* coarse, int ncell_coarse, int D, hipStream_t s);

}  // namespace vps
