// Launchers of the plane-streaming 3D kernels (operator, residual, restriction).
#include "kernels.h"
#include "launch.h"
#include "stream3.h"

namespace vps {

namespace {

// Workgroups wanted per launch: several per CU on the 256 CUs, so that the
// chunks along z are long enough for the halo cell layer to stay cheap.
constexpr int kStreamTarget = 3072;

template <typename T, int KIND, int K>
hipError_t go_stream(const StreamLaunch& L, hipStream_t s) {
  using S = StreamShape<KIND, K>;
  static_assert(S::LDS_ELEMS * sizeof(T) <= 65536, "stream tile does not fit the workgroup LDS");
  static_assert(sizeof(StreamArgs<T, KIND, K>) <= 4096, "kernel arguments exceed 4 KiB");
  // cells per direction of the grid the tiles and chunks are cut from (the coarse grid for the prolongation)
  const int n = L.ncell_out;
  if (n < 1) return hipErrorInvalidValue;
  StreamArgs<T, KIND, K> a;
  a.in = (const T*)L.in;
  a.b = (const T*)L.b;
  a.out = (T*)L.out;
  a.n1_in = L.n1_in;
  a.n1_out = L.n1_out;
  a.ncz = n;
  a.tiles_x = (n + S::TX - 1) / S::TX;
  a.tiles_y = (n + S::TY - 1) / S::TY;
  const long long xy = (long long)a.tiles_x * a.tiles_y;
  const long long want_chunks = (kStreamTarget + xy - 1) / xy;
  int cz = (int)((n + want_chunks - 1) / want_chunks);
  if (cz < 2) cz = 2;
  if (cz > n) cz = n;
  a.cz = cz;
  const long long chunks = (n + cz - 1) / cz;
  const long long nb = xy * chunks;
  if (nb >= (1LL << 31)) return hipErrorInvalidValue;
  // plane sizes and offsets are formed in 32-bit inside the kernel
  if ((long long)L.n1_in * L.n1_in >= (1LL << 31) || (long long)L.n1_out * L.n1_out >= (1LL << 31))
    return hipErrorInvalidValue;
  a.nblocks = (unsigned)nb;
  constexpr int ZW = S::ZIN + 1;
  if constexpr (S::OP) {
    // Z0, Z1: the cell mass and stiffness matrices ((K+1) x (K+1)); G0, G1: the period rows,
    // whose vertex row (row 0) holds the diagonal summed over both cells at window position K
    for (int r = 0; r <= K; ++r)
      for (int c = r; c <= K; ++c) {
        a.cm[cell_sym_idx(r, c, K)] = (T)L.Z0[r * ZW + c];
        a.ck[cell_sym_idx(r, c, K)] = (T)L.Z1[r * ZW + c];
      }
    a.mvv = (T)L.G0[K];
    a.kvv = (T)L.G1[K];
    a.pt[0] = T(0);
  } else {
    // p[f][c], f = 0..K: the prolongation's period rows (G0, 2K x (K+1)), or the restriction's
    // z table transposed (Z0[c][f] for fine planes f < 2K of a coarse cell)
    for (int f = 0; f <= K; ++f)
      for (int c = 0; c <= K; ++c)
        a.pt[f * (K + 1) + c] = S::PR ? (T)L.G0[f * (K + 1) + c] : (T)L.Z0[c * ZW + f];
    a.cm[0] = a.ck[0] = a.mvv = a.kvv = T(0);
  }
  const unsigned grid = (unsigned)((nb + kXcd - 1) / kXcd * kXcd);
  stream3_kernel<T, KIND, K><<<grid, kBlock, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace

template <typename T, int K>
hipError_t launch_stream_operator(const StreamLaunch& L, hipStream_t s) {
  return L.b ? go_stream<T, STREAM_RESIDUAL, K>(L, s) : go_stream<T, STREAM_OPERATOR, K>(L, s);
}
template <typename T, int K>
hipError_t launch_stream_restrict(const StreamLaunch& L, hipStream_t s) {
  return go_stream<T, STREAM_RESTRICT, K>(L, s);
}
template <typename T, int K>
hipError_t launch_stream_prolong(const StreamLaunch& L, hipStream_t s) {
  return go_stream<T, STREAM_PROLONG, K>(L, s);
}

#define VPS_STREAM_INST(T, K)                                                           \
  template hipError_t launch_stream_operator<T, K>(const StreamLaunch&, hipStream_t);  \
  template hipError_t launch_stream_restrict<T, K>(const StreamLaunch&, hipStream_t);  \
  template hipError_t launch_stream_prolong<T, K>(const StreamLaunch&, hipStream_t);
VPS_STREAM_INST(double, 1) VPS_STREAM_INST(double, 2) VPS_STREAM_INST(double, 3) VPS_STREAM_INST(double, 4)
VPS_STREAM_INST(double, 5)
VPS_STREAM_INST(float, 1) VPS_STREAM_INST(float, 2) VPS_STREAM_INST(float, 3) VPS_STREAM_INST(float, 4)
VPS_STREAM_INST(float, 5)

}  // namespace vps
