// Launcher of the patch smoother kernel for one degree (VPS_PATCH_K), included
// by patch_k<K>.hip so that the degrees compile in parallel.
#include <algorithm>

#include "kernels.h"
#include "patch_wave.h"
#include "patch_pair.h"
#include "patch_row2.h"
#include "patch_row3.h"
#include "patch_row5.h"
#include "patch_big.h"
#include "patch_solve.h"
#include "launch.h"

namespace vps {

namespace {

template <typename T, int K, int D, int COEF, int PB>
hipError_t go_patch(const PatchArgs<T, K>& a, hipStream_t s) {
  using Sh = PatchKernelShape<T, K, D, COEF, PB>;
  if constexpr (Sh::LDS_BYTES + 4096 > 65536) {
    return hipErrorInvalidValue;  // shape does not fit the 64 KiB workgroup LDS limit
  } else {
    dim3 grid((a.np[0] + PB - 1) / PB, a.np[1], D == 3 ? a.np[2] : 1);
    patch_color_kernel<T, K, D, COEF, PB><<<grid, kBlock, 0, s>>>(a);
    return hipGetLastError();
  }
}

template <typename T, int K, int D, int COEF>
hipError_t go_patch_pb(const PatchArgs<T, K>& a, int pb, hipStream_t s) {
  switch (pb) {
    case 1: return go_patch<T, K, D, COEF, 1>(a, s);
    case 2: return go_patch<T, K, D, COEF, 2>(a, s);
    case 4: return go_patch<T, K, D, COEF, 4>(a, s);
    default: return hipErrorInvalidValue;
  }
}

// Arguments of the row kernels (groups of G patches of one color, packed along
// the rows of patches when a row holds at least G of them); false if the
// group decomposition's exact divisions do not hold.
template <typename T, int K, int G>
bool fill_row_args(const PatchArgs<T, K>& a, const PatchLaunch& L, unsigned vec_bytes, Row3Args<T, K>* w) {
  w->u = a.u;
  w->b = a.b;
  w->n1 = a.n1;
  for (int e = 0; e < 3; ++e) {
    w->v0[e] = a.v0[e];
    w->np[e] = a.np[e];
  }
  w->ngx = (a.np[0] + G - 1) / G;
  const unsigned long long npatch = (unsigned long long)a.np[0] * (unsigned)a.np[1] * (unsigned)a.np[2];
  w->packed = a.np[0] >= G ? 1 : 0;
  const unsigned long long ng = w->packed ? (npatch + G - 1) / G
                                          : (unsigned long long)w->ngx * (unsigned)a.np[1] * (unsigned)a.np[2];
  // the group decomposition divides numbers below ngroups by ngx and np[1] (row groups) or
  // numbers below npatch by np[0] and np[1] (packed)
  if (ng * (unsigned)w->ngx >= (1ull << 32) || ng * (unsigned)a.np[1] >= (1ull << 32) ||
      npatch * (unsigned)a.np[0] >= (1ull << 32) || npatch * (unsigned)a.np[1] >= (1ull << 32))
    return false;
  w->ngroups = (unsigned)ng;
  w->npatch = (unsigned)npatch;
  w->vec_bytes = vec_bytes;
  w->magic_g = magic_of((unsigned)w->ngx);
  w->magic_x = magic_of((unsigned)a.np[0]);
  w->magic_y = magic_of((unsigned)a.np[1]);
  PatchBand<T, K> band;
  if (!make_band<T, K>(L.M[0], L.Kst[0], &band)) return false;
  make_sym_band<T, K>(band, &w->band);
  for (int i = 0; i < K * K; ++i) w->f.Te[i] = (T)L.Te[i];
  for (int i = 0; i < (K - 1) * (K - 1); ++i) w->f.To[i] = (T)L.To[i];
  for (int i = 0; i < 2 * K - 1; ++i) w->lam[i] = (T)L.lam_int[i];
  return true;
}

}  // namespace

template <typename T, int K, int D>
hipError_t launch_patch_color(const PatchLaunch& L, hipStream_t s) {
  static_assert(sizeof(PatchArgs<T, K>) <= 4096, "kernel arguments exceed 4 KiB");
  using PM = PatchMats<T, K>;
  constexpr int P = PM::P, Q = PM::Q;
  PatchArgs<T, K> a;
  a.u = (T*)L.u;
  a.b = (const T*)L.b;
  a.rho = (const T*)L.rho;
  a.scal = L.scal;
  a.n1 = L.n1;
  a.ncell = L.ncell;
  const int N = L.ncell;
  for (int e = 0; e < 3; ++e) {
    if (e >= D) { a.v0[e] = 1; a.np[e] = 1; continue; }
    const int bit = (L.color >> e) & 1;
    int v0 = bit ? 1 : 2, vlast = N - 1;
    if (e == D - 1 && L.vhi > 0) {  // one batch: the vertex layers [vlo, vhi] of the slowest direction
      v0 = L.vlo + (((L.vlo & 1) != bit) ? 1 : 0);
      vlast = std::min(L.vhi, N - 1);
    }
    a.v0[e] = v0;
    a.np[e] = (v0 <= vlast) ? (vlast - v0) / 2 + 1 : 0;
    if (a.np[e] == 0) return hipSuccess;  // no patch of this color
  }
  for (int h = 0; h < 2; ++h)
    for (int i = 0; i < Q * P; ++i) {
      a.m.M[h][i] = L.M[h] ? (T)L.M[h][i] : T(0);
      a.m.Kst[h][i] = L.Kst[h] ? (T)L.Kst[h][i] : T(0);
    }
  for (int i = 0; i < Q * Q; ++i) a.m.T1[i] = (T)L.T1[i];
  for (int i = 0; i < Q; ++i) a.m.lam[i] = (T)L.lam[i];
  // 2D, rho = 1: a row of patches per wave from 64 cells per direction (measured
  // faster than the LDS-staged kernel there for every degree 2..5; below, both
  // are launch-latency bound)
  const bool row2 = L.row2 == 1 || (L.row2 == 0 && N >= 64);
  if (D == 2 && L.coef == 0 && L.pb == 0 && L.Te && L.lam_int && row2) {
    if constexpr (K >= 2 && K <= 5) {  // a row of patches per wave
      static_assert(sizeof(RowArgs<T, K>) <= 4096, "kernel arguments exceed 4 KiB");
      using R = RowShape<K>;
      RowArgs<T, K> w;
      w.u = a.u;
      w.b = a.b;
      w.n1 = a.n1;
      for (int e = 0; e < 2; ++e) {
        w.v0[e] = a.v0[e];
        w.np[e] = a.np[e];
      }
      w.ngx = (a.np[0] + R::G - 1) / R::G;
      const unsigned long long ng = (unsigned long long)w.ngx * (unsigned)a.np[1];
      if (ng * (unsigned)w.ngx >= (1ull << 32)) return hipErrorInvalidValue;  // exact division by ngx
      w.ngroups = (unsigned)ng;
      const unsigned long long vbytes = (unsigned long long)a.n1 * a.n1 * sizeof(T);
      if (vbytes >= (1ull << 32)) return hipErrorInvalidValue;  // buffer offsets are 32-bit
      w.vec_bytes = (unsigned)vbytes;
      w.magic_g = magic_of((unsigned)w.ngx);
      if (!make_band<T, K>(L.M[0], L.Kst[0], &w.band)) return hipErrorInvalidValue;
      for (int i = 0; i < K * K; ++i) w.f.Te[i] = (T)L.Te[i];
      for (int i = 0; i < (K - 1) * (K - 1); ++i) w.f.To[i] = (T)L.To[i];
      for (int i = 0; i < Q; ++i) w.lam[i] = (T)L.lam_int[i];
      const unsigned grid = (w.ngroups + kXcd - 1) / kXcd * kXcd;  // a multiple of the XCD count
      patch_row2_kernel<T, K><<<grid, 64, 0, s>>>(w);
      return hipGetLastError();
    }
  }
  if (D == 3 && L.coef == 0 && L.pb == 0 && L.order == 0 && L.Te && L.lam_int) {
    if constexpr (K == 5) {
      if (L.ppw == 3) {  // a row of patches per workgroup of two waves
        static_assert(sizeof(Row3Args<T, K>) <= 4096, "kernel arguments exceed 4 KiB");
        const unsigned long long vbytes = (unsigned long long)a.n1 * a.n1 * a.n1 * sizeof(T);
        if (vbytes >= (1ull << 32)) return hipErrorInvalidValue;  // buffer offsets are 32-bit
        Row3Args<T, K> w;
        if (!fill_row_args<T, K, Row5Shape<K>::G>(a, L, (unsigned)vbytes, &w)) return hipErrorInvalidValue;
        const unsigned grid = (w.ngroups + kXcd - 1) / kXcd * kXcd;  // a multiple of the XCD count
        patch_row5_kernel<T, K><<<grid, 128, 0, s>>>(w);
        return hipGetLastError();
      }
      // one patch per wave, the interior lines in passes of 64
      static_assert(sizeof(BigArgs<T, K>) <= 4096, "kernel arguments exceed 4 KiB");
      BigArgs<T, K> w;
      w.u = a.u;
      w.b = a.b;
      w.n1 = a.n1;
      for (int e = 0; e < 3; ++e) {
        w.v0[e] = a.v0[e];
        w.np[e] = a.np[e];
      }
      w.npatch = (unsigned)a.np[0] * (unsigned)a.np[1] * (unsigned)a.np[2];
      if ((unsigned long long)w.npatch * (unsigned)a.np[0] >= (1ull << 32) ||
          (unsigned long long)w.npatch * (unsigned)a.np[1] >= (1ull << 32))
        return hipErrorInvalidValue;  // exact division by np[0] and np[1]
      const unsigned long long vbytes = (unsigned long long)a.n1 * a.n1 * a.n1 * sizeof(T);
      if (vbytes >= (1ull << 32)) return hipErrorInvalidValue;  // buffer offsets are 32-bit
      w.vec_bytes = (unsigned)vbytes;
      w.magic_x = magic_of((unsigned)a.np[0]);
      w.magic_y = magic_of((unsigned)a.np[1]);
      PatchBand<T, K> band;
      if (!make_band<T, K>(L.M[0], L.Kst[0], &band)) return hipErrorInvalidValue;
      make_sym_band<T, K>(band, &w.band);
      for (int i = 0; i < K * K; ++i) w.f.Te[i] = (T)L.Te[i];
      for (int i = 0; i < (K - 1) * (K - 1); ++i) w.f.To[i] = (T)L.To[i];
      for (int i = 0; i < Q; ++i) w.lam[i] = (T)L.lam_int[i];
      const unsigned grid = (w.npatch + kXcd - 1) / kXcd * kXcd;  // a multiple of the XCD count
      patch_big3_kernel<T, K><<<grid, 64, 0, s>>>(w);
      return hipGetLastError();
    }
  }
  if (D == 3 && L.coef == 0 && L.pb == 0) {
    if constexpr (K >= 2 && K <= 4) {  // (2K-1)^2 interior lines must fit the 64 lanes of a wave
      static_assert(sizeof(WaveArgs<T, K>) <= 4096, "kernel arguments exceed 4 KiB");
      static_assert(sizeof(PairArgs<T, K>) <= 4096, "kernel arguments exceed 4 KiB");
      const unsigned long long vbytes = (unsigned long long)a.n1 * a.n1 * a.n1 * sizeof(T);
      if (vbytes >= (1ull << 32)) return hipErrorInvalidValue;  // buffer offsets are 32-bit
      if (L.ppw == 3) {
        if (L.order != 0) return hipErrorInvalidValue;  // rows are visited in lexicographic order only
        static_assert(sizeof(Row3Args<T, K>) <= 4096, "kernel arguments exceed 4 KiB");
        Row3Args<T, K> w;
        if (!fill_row_args<T, K, Row3Shape<K>::G>(a, L, (unsigned)vbytes, &w)) return hipErrorInvalidValue;
        const unsigned grid = (w.ngroups + kXcd - 1) / kXcd * kXcd;  // a multiple of the XCD count
        patch_row3_kernel<T, K><<<grid, 64, 0, s>>>(w);
        return hipGetLastError();
      }
      if (L.ppw == 2) {
        if (L.order != 0) return hipErrorInvalidValue;  // pairs are visited in lexicographic order only
        PairArgs<T, K> w;
        w.u = a.u;
        w.b = a.b;
        w.n1 = a.n1;
        for (int e = 0; e < 3; ++e) {
          w.v0[e] = a.v0[e];
          w.np[e] = a.np[e];
        }
        w.ngx = (a.np[0] + 1) / 2;
        const unsigned long long ng = (unsigned long long)w.ngx * (unsigned)a.np[1] * (unsigned)a.np[2];
        // the pair decomposition divides numbers below ngroups by ngx and np[1]
        if (ng * (unsigned)w.ngx >= (1ull << 32) || ng * (unsigned)a.np[1] >= (1ull << 32)) return hipErrorInvalidValue;
        w.ngroups = (unsigned)ng;
        w.vec_bytes = (unsigned)vbytes;
        w.magic_g = magic_of((unsigned)w.ngx);
        w.magic_y = magic_of((unsigned)a.np[1]);
        if (!make_band<T, K>(L.M[0], L.Kst[0], &w.band)) return hipErrorInvalidValue;
        for (int i = 0; i < K * K; ++i) w.f.Te[i] = (T)L.Te[i];
        for (int i = 0; i < (K - 1) * (K - 1); ++i) w.f.To[i] = (T)L.To[i];
        for (int i = 0; i < Q; ++i) w.lam[i] = (T)L.lam_int[i];
        const unsigned grid = (w.ngroups + kXcd - 1) / kXcd * kXcd;  // a multiple of the XCD count
        patch_pair3_kernel<T, K><<<grid, 64, 0, s>>>(w);
        return hipGetLastError();
      }
      WaveArgs<T, K> w;
      w.u = a.u;
      w.b = a.b;
      w.n1 = a.n1;
      for (int e = 0; e < 3; ++e) {
        w.v0[e] = a.v0[e];
        w.np[e] = a.np[e];
      }
      w.npatch = (unsigned)a.np[0] * (unsigned)a.np[1] * (unsigned)a.np[2];
      // the patch decomposition divides numbers below npatch by np[0] and np[1]
      if ((unsigned long long)w.npatch * (unsigned)a.np[0] >= (1ull << 32) ||
          (unsigned long long)w.npatch * (unsigned)a.np[1] >= (1ull << 32))
        return hipErrorInvalidValue;
      w.vec_bytes = (unsigned)vbytes;
      w.magic_x = magic_of((unsigned)a.np[0]);
      w.magic_y = magic_of((unsigned)a.np[1]);
      if (!make_band<T, K>(L.M[0], L.Kst[0], &w.band)) return hipErrorInvalidValue;
      for (int i = 0; i < K * K; ++i) w.f.Te[i] = (T)L.Te[i];
      for (int i = 0; i < (K - 1) * (K - 1); ++i) w.f.To[i] = (T)L.To[i];
      for (int i = 0; i < Q; ++i) w.lam[i] = (T)L.lam_int[i];
      // one wave per patch; the grid is padded to a multiple of the XCD count
      w.order = L.order;
      w.cover_log2 = 0;
      w.tiles_x = w.tiles_y = 1;
      if (L.order <= 1) {
        w.nslots = w.npatch;
      } else if (L.order == 2) {
        const int m = std::max(a.np[0], std::max(a.np[1], a.np[2]));
        while ((1 << w.cover_log2) < m) ++w.cover_log2;
        if (w.cover_log2 > 10) return hipErrorInvalidValue;
        w.nslots = 1u << (3 * w.cover_log2);
      } else if (L.order == 3) {
        w.tiles_x = (a.np[0] + 3) / 4;
        w.tiles_y = (a.np[1] + 3) / 4;
        const unsigned long long slots = 64ull * w.tiles_x * w.tiles_y * ((a.np[2] + 3) / 4);
        if (slots >= (1ull << 31)) return hipErrorInvalidValue;
        w.nslots = (unsigned)slots;
      } else {
        return hipErrorInvalidValue;
      }
      const unsigned grid = (w.nslots + kXcd - 1) / kXcd * kXcd;
      patch_wave3_kernel<T, K><<<grid, 64, 0, s>>>(w);
      return hipGetLastError();
    }
  }
  const int pb = L.pb > 0 ? L.pb : default_patches_per_block(K, D, L.coef, sizeof(T) == 8);  // 0, -1: automatic
  switch (L.coef) {
    case 0: return go_patch_pb<T, K, D, 0>(a, pb, s);
    case 1: return go_patch_pb<T, K, D, 1>(a, pb, s);
    case 2: return go_patch_pb<T, K, D, 2>(a, pb, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int K>
hipError_t launch_patch_solve(const PatchLaunch& L, const void* r, hipStream_t s) {
  if constexpr (K < 2 || K > 4) {
    return hipErrorInvalidValue;  // even/odd FDM needs K >= 2; one wave per patch needs (2K-1)^2 <= 64
  } else {
    static_assert(sizeof(SolveArgs<T, K>) <= 4096, "kernel arguments exceed 4 KiB");
    constexpr int Q = 2 * K - 1;
    if (!L.Te || !L.To || !L.lam_int) return hipErrorInvalidValue;
    SolveArgs<T, K> w;
    w.u = (T*)L.u;
    w.r = (const T*)r;
    w.n1 = L.n1;
    const int N = L.ncell;
    for (int e = 0; e < 3; ++e) {
      const int v0 = ((L.color >> e) & 1) ? 1 : 2;
      w.v0[e] = v0;
      w.np[e] = (v0 <= N - 1) ? (N - 1 - v0) / 2 + 1 : 0;
      if (w.np[e] == 0) return hipSuccess;  // no patch of this color
    }
    w.npatch = (unsigned)w.np[0] * (unsigned)w.np[1] * (unsigned)w.np[2];
    if ((unsigned long long)w.npatch * (unsigned)w.np[0] >= (1ull << 32) ||
        (unsigned long long)w.npatch * (unsigned)w.np[1] >= (1ull << 32))
      return hipErrorInvalidValue;
    const unsigned long long vbytes = (unsigned long long)L.n1 * L.n1 * L.n1 * sizeof(T);
    if (vbytes >= (1ull << 32)) return hipErrorInvalidValue;  // buffer offsets are 32-bit
    w.vec_bytes = (unsigned)vbytes;
    w.magic_x = magic_of((unsigned)w.np[0]);
    w.magic_y = magic_of((unsigned)w.np[1]);
    for (int i = 0; i < K * K; ++i) w.f.Te[i] = (T)L.Te[i];
    for (int i = 0; i < (K - 1) * (K - 1); ++i) w.f.To[i] = (T)L.To[i];
    for (int i = 0; i < Q; ++i) w.lam[i] = (T)L.lam_int[i];
    const unsigned grid = (w.npatch + kXcd - 1) / kXcd * kXcd;
    patch_solve3_kernel<T, K><<<grid, 64, 0, s>>>(w);
    return hipGetLastError();
  }
}

template hipError_t launch_patch_solve<double, VPS_PATCH_K>(const PatchLaunch&, const void*, hipStream_t);
template hipError_t launch_patch_solve<float, VPS_PATCH_K>(const PatchLaunch&, const void*, hipStream_t);
template hipError_t launch_patch_color<double, VPS_PATCH_K, 2>(const PatchLaunch&, hipStream_t);
template hipError_t launch_patch_color<double, VPS_PATCH_K, 3>(const PatchLaunch&, hipStream_t);
template hipError_t launch_patch_color<float, VPS_PATCH_K, 2>(const PatchLaunch&, hipStream_t);
template hipError_t launch_patch_color<float, VPS_PATCH_K, 3>(const PatchLaunch&, hipStream_t);

}  // namespace vps
