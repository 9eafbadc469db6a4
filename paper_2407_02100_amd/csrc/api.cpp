// C ABI of libvps: context, level set-up, smoother/V-cycle/CG drivers.
// Declarations and the contract of every entry point are in include/vps.h.
#include "vps.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fe_host.h"
#include "launch.h"
#include "mlp_launch.h"

using vps::Mat;

namespace {

struct Level {
  int ncell = 0, n1 = 0;
  size_t nodes = 0;
  long long npatch = 0;
  double h = 0.0;
  void* u = nullptr;  // V-cycle work vectors in the V-cycle dtype
  void* b = nullptr;
  void* r = nullptr;
  void* sep_r = nullptr;  // separated smoother: global residual of a color step (FP64-sized, either dtype)
  double* rho64 = nullptr;  // per-cell coefficient
  float* rho32 = nullptr;
  float* scal = nullptr;    // learned per-patch eigenmode factors
  double* binv = nullptr;   // exact local solvers: per patch A_j(rho)^{-1}, 27 x 27 FP64 (Q2, 3D)
  // 2-cell patch: interior rows (q x p) of mass/stiffness; halves per cell
  Mat Mfull, Kfull, Mh[2], Kh[2];
  Mat T1;                   // FDM eigenvectors (q x q)
  std::vector<double> lam;  // FDM eigenvalues (q)
  std::vector<double> lam_int;  // the same in the even/odd mode order
  Mat Te, To;               // even/odd blocks of T1 (symmetric / antisymmetric modes)
  Mat opM, opK;             // operator tile blocks
  Mat restrictG;            // transfer tile: this level -> level-1
  Mat prolongG;             // transfer tile: level-1 -> this level
  Mat Mc, Kc;               // cell matrices (h-scaled)
  // plane-streaming kernels (3D): period rows of the 1D operators and z cell tables
  Mat sG0, sG1, sZ0, sZ1;   // operator: mass / stiffness, K x (2K+1) and (K+1) x (K+1)
  Mat rG, rZ;               // restriction to level-1: K x (4K+1) and (K+1) x (2K+1)
  Mat pG;                   // prolongation from level-1: 2K x (K+1) (period rows and z cell table)
};

enum Phase { PH_SMOOTH, PH_RESIDUAL, PH_RESTRICT, PH_PROLONG, PH_COARSE, PH_CG_OP, PH_CG_VEC };

// Event pairs recorded around phases; resolved (synchronously) by flush().
struct PhaseTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec {
    int phase, level;
    hipEvent_t a, b;
    long long sweeps;
  };
  std::vector<Rec> recs;
  vps_timing tot{};
};

}  // namespace

struct vps_context {
  vps_config cfg{};
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<Level> lv;
  // coarse solver: FDM of the coarse grid (rho = 1) ...
  int cn0 = 0;
  void* cT0[2] = {nullptr, nullptr};   // [0] FP64, [1] FP32
  void* clam0[2] = {nullptr, nullptr};
  // ... or a dense inverse (cell coefficient)
  void* cAinv[2] = {nullptr, nullptr};
  int* cfree = nullptr;
  int cnfree = 0;
  bool coarse_ok = false;  // a coarse solver exists for level 0
  bool coef_set = false;
  std::vector<long long> fallback;  // per level: patches whose learned scaling fell back to 1
  // CG work vectors (FP64, finest level)
  double* cg_r = nullptr;
  double* cg_p = nullptr;
  double* cg_q = nullptr;
  double* cg_z = nullptr;
  double* partial = nullptr;
  double* dscal = nullptr;
  double* hscal = nullptr;  // pinned host
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // MLP work
  vps::MlpWork mlp;
  PhaseTimer timer;
  // V-cycles captured as HIP graphs, one per (finest-level input, output) pair
  struct VcycleGraph {
    const void* b;
    void* u;
    hipGraphExec_t exec;
  };
  std::vector<VcycleGraph> graphs;
  hipStream_t capture_stream = nullptr;  // created on the first capture
  bool graphs_failed = false;            // a capture failed: launch kernel by kernel from then on
};

namespace {

constexpr int kMaxDenseCoarse = 4096;

// message of the last failed vps_create (no context exists then)
thread_local std::string g_create_error;

const char* kStatusText[] = {"ok",           "invalid argument", "unsupported configuration",
                             "HIP error",    "out of device memory", "not converged",
                             "non-finite value", "invalid state"};

vps_status fail(vps_context* c, vps_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

vps_status hip_fail(vps_context* c, hipError_t e, const char* what) {
  if (c) c->err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? VPS_E_NOMEM : VPS_E_HIP;
}

#define VPS_HIP(ctx, call)                                      \
  do {                                                          \
    hipError_t e_ = (call);                                     \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #call);    \
  } while (0)

template <typename T, typename F>
hipError_t dispatch_kd(int k, int d, F& f) {
#define VPS_KD(KK, DD) \
  if (k == KK && d == DD) return f.template operator()<T, KK, DD>();
  VPS_KD(1, 2) VPS_KD(1, 3) VPS_KD(2, 2) VPS_KD(2, 3) VPS_KD(3, 2) VPS_KD(3, 3) VPS_KD(4, 2) VPS_KD(4, 3)
  VPS_KD(5, 2) VPS_KD(5, 3)
#undef VPS_KD
  return hipErrorInvalidValue;
}

template <typename F>
hipError_t dispatch_tkd(vps_dtype t, int k, int d, F&& f) {
  if (t == VPS_F64) return dispatch_kd<double>(k, d, f);
  return dispatch_kd<float>(k, d, f);
}

template <typename T, typename F>
hipError_t dispatch_k(int k, F& f) {
  switch (k) {
    case 1: return f.template operator()<T, 1>();
    case 2: return f.template operator()<T, 2>();
    case 3: return f.template operator()<T, 3>();
    case 4: return f.template operator()<T, 4>();
    case 5: return f.template operator()<T, 5>();
  }
  return hipErrorInvalidValue;
}

template <typename F>
hipError_t dispatch_tk(vps_dtype t, int k, F&& f) {
  if (t == VPS_F64) return dispatch_k<double>(k, f);
  return dispatch_k<float>(k, f);
}

hipError_t timer_flush(vps_context* c);

// Start a phase; returns its record index or -1 when timing is off.
int tbegin(vps_context* c, int phase, int level, long long sweeps = 0) {
  PhaseTimer& T = c->timer;
  if (!T.on) return -1;
  if (T.used + 2 > T.pool.size()) {
    if (T.used >= 4096) {
      if (timer_flush(c) != hipSuccess) return -1;
    } else {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        T.pool.push_back(e);
      }
    }
  }
  PhaseTimer::Rec r{phase, level, T.pool[T.used], T.pool[T.used + 1], sweeps};
  T.used += 2;
  if (hipEventRecord(r.a, c->stream) != hipSuccess) return -1;
  T.recs.push_back(r);
  return (int)T.recs.size() - 1;
}

void tend(vps_context* c, int idx) {
  if (idx < 0) return;
  (void)hipEventRecord(c->timer.recs[idx].b, c->stream);
}

hipError_t timer_flush(vps_context* c) {
  PhaseTimer& T = c->timer;
  if (T.recs.empty()) return hipSuccess;
  hipError_t e = hipEventSynchronize(T.recs.back().b);
  if (e != hipSuccess) return e;
  for (const auto& r : T.recs) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return e;
    const double s = ms * 1e-3;
    const int l = r.level < VPS_MAX_LEVELS ? r.level : VPS_MAX_LEVELS - 1;
    switch (r.phase) {
      case PH_SMOOTH: T.tot.smooth_s[l] += s; T.tot.smooth_sweeps[l] += r.sweeps; break;
      case PH_RESIDUAL: T.tot.residual_s[l] += s; break;
      case PH_RESTRICT: T.tot.restrict_s[l] += s; break;
      case PH_PROLONG: T.tot.prolong_s[l] += s; break;
      case PH_COARSE: T.tot.coarse_s += s; break;
      case PH_CG_OP: T.tot.cg_operator_s += s; break;
      default: T.tot.cg_vector_s += s; break;
    }
  }
  T.recs.clear();
  T.used = 0;
  return hipSuccess;
}

size_t esize(vps_dtype t) { return t == VPS_F64 ? sizeof(double) : sizeof(float); }

int ipow(int a, int d) {
  int r = 1;
  for (int i = 0; i < d; ++i) r *= a;
  return r;
}

void build_level(Level& L, int k, int d, int ncell) {
  L.ncell = ncell;
  L.n1 = k * ncell + 1;
  L.nodes = 1;
  for (int e = 0; e < d; ++e) L.nodes *= (size_t)L.n1;
  L.npatch = 1;
  for (int e = 0; e < d; ++e) L.npatch *= (long long)(ncell - 1);
  L.h = 1.0 / ncell;
  const int p = 2 * k + 1, q = 2 * k - 1;
  Mat Mp, Kp;
  vps::assemble_1d(k, 2, L.h, &Mp, &Kp);
  L.Mfull.assign(q * p, 0.0);
  L.Kfull.assign(q * p, 0.0);
  for (int o = 0; o < q; ++o)
    for (int i = 0; i < p; ++i) {
      L.Mfull[o * p + i] = Mp[(o + 1) * p + i];
      L.Kfull[o * p + i] = Kp[(o + 1) * p + i];
    }
  for (int h = 0; h < 2; ++h) {
    const double w[2] = {h == 0 ? 1.0 : 0.0, h == 1 ? 1.0 : 0.0};
    Mat Mh, Kh;
    vps::assemble_1d(k, 2, L.h, &Mh, &Kh, w);
    L.Mh[h].assign(q * p, 0.0);
    L.Kh[h].assign(q * p, 0.0);
    for (int o = 0; o < q; ++o)
      for (int i = 0; i < p; ++i) {
        L.Mh[h][o * p + i] = Mh[(o + 1) * p + i];
        L.Kh[h][o * p + i] = Kh[(o + 1) * p + i];
      }
  }
  Mat Mi(q * q), Ki(q * q);
  for (int o = 0; o < q; ++o)
    for (int j = 0; j < q; ++j) {
      Mi[o * q + j] = Mp[(o + 1) * p + j + 1];
      Ki[o * q + j] = Kp[(o + 1) * p + j + 1];
    }
  vps::gen_eig(q, Mi, Ki, &L.T1, &L.lam);
  std::vector<int> order;
  if (!vps::fdm_even_odd(q, L.T1, &L.Te, &L.To, &order)) {
    L.Te.clear();  // no even/odd structure: the one-patch-per-wave kernels are not used
  } else {
    L.lam_int.resize(q);
    for (int j = 0; j < q; ++j) L.lam_int[j] = L.lam[order[j]];
  }
  // operator tile
  {
    const int TC = vps::op_tc(k, d);
    Mat M, K;
    vps::assemble_1d(k, TC + 2, L.h, &M, &K);
    const int n = k * (TC + 2) + 1, NO = k * TC, NI = k * (TC + 1) + 1;
    L.opM.assign(NO * NI, 0.0);
    L.opK.assign(NO * NI, 0.0);
    for (int o = 0; o < NO; ++o)
      for (int i = 0; i < NI; ++i) {
        L.opM[o * NI + i] = M[(k + o) * n + i];
        L.opK[o * NI + i] = K[(k + o) * n + i];
      }
  }
  // transfer tiles (used only when a coarser level exists)
  {
    const int TC = vps::restrict_tc(k, d);
    const int nc = TC + 2;
    Mat P1;
    vps::prolongation_1d(k, nc, &P1);
    const int ncn = k * nc + 1, NO = k * TC, NI = 2 * k * (TC + 1) + 1;
    L.restrictG.assign(NO * NI, 0.0);
    for (int o = 0; o < NO; ++o)
      for (int i = 0; i < NI; ++i) L.restrictG[o * NI + i] = P1[(size_t)i * ncn + k + o];
  }
  {
    const int TC = vps::prolong_tc(k, d);
    const int nc = TC + 1;
    Mat P1;
    vps::prolongation_1d(k, nc, &P1);
    const int ncn = k * nc + 1, NO = 2 * k * TC, NI = k * TC + 1;
    L.prolongG.assign(NO * NI, 0.0);
    for (int o = 0; o < NO; ++o)
      for (int i = 0; i < NI; ++i) L.prolongG[o * NI + i] = P1[(size_t)o * ncn + i];
  }
  Mat Mr, Kr;
  vps::reference_matrices(k, &Mr, &Kr);
  L.Mc.resize(Mr.size());
  L.Kc.resize(Kr.size());
  for (size_t i = 0; i < Mr.size(); ++i) {
    L.Mc[i] = L.h * Mr[i];
    L.Kc[i] = Kr[i] / L.h;
  }
  // streaming tables: rows k..2k-1 of the 1D operators of a two-cell mesh (the
  // vertex row and the interior rows of a cell, translation invariant), and the
  // 1D prolongation block of coarse cell 1 of a two-cell coarse mesh
  {
    Mat M, K;
    vps::assemble_1d(k, 2, L.h, &M, &K);
    const int n = 2 * k + 1, W = 2 * k + 1;
    L.sG0.assign(k * W, 0.0);
    L.sG1.assign(k * W, 0.0);
    for (int j = 0; j < k; ++j)
      for (int i = 0; i < W; ++i) {
        L.sG0[j * W + i] = M[(k + j) * n + i];
        L.sG1[j * W + i] = K[(k + j) * n + i];
      }
    L.sZ0 = L.Mc;
    L.sZ1 = L.Kc;
  }
  {
    Mat P1;
    vps::prolongation_1d(k, 2, &P1);
    const int ncn = 2 * k + 1, W = 4 * k + 1, ZW = 2 * k + 1;
    L.rG.assign(k * W, 0.0);
    for (int j = 0; j < k; ++j)
      for (int i = 0; i < W; ++i) L.rG[j * W + i] = P1[(size_t)i * ncn + k + j];
    L.rZ.assign((k + 1) * ZW, 0.0);
    for (int i = 0; i <= k; ++i)
      for (int l = 0; l < 2 * k; ++l) L.rZ[i * ZW + l] = P1[(size_t)l * ncn + i];
    L.pG.assign(2 * k * (k + 1), 0.0);
    for (int j = 0; j < 2 * k; ++j)
      for (int i = 0; i <= k; ++i) L.pG[j * (k + 1) + i] = P1[(size_t)j * ncn + i];
  }
}

template <typename T>
hipError_t upload(const std::vector<double>& src, void** dst, hipStream_t s) {
  std::vector<T> tmp(src.begin(), src.end());
  hipError_t e = hipMalloc(dst, tmp.size() * sizeof(T));
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(*dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

bool level_ok(const vps_context* c, int l) { return c && l >= 0 && l < (int)c->lv.size(); }

// cells per direction from which the plane-streaming kernels are used
// the two-patches-per-wave smoother kernel: 3D, rho = 1, degree 2..4, combined
// algorithm, default dispatch order, automatic workgroup shape
bool pair_kernel_applies(const vps_config& C) {
  return C.dim == 3 && C.coef == VPS_COEF_CONST && C.degree >= 2 && C.degree <= 4 &&
         C.algorithm == VPS_ALG_COMBINED && C.patch_order == 0 && C.patches_per_block == 0;
}
// the row-of-patches smoother kernels: as the pair kernel, degrees 2..5 (degree 5: two waves per row)
bool row_kernel_applies(const vps_config& C) {
  return C.dim == 3 && C.coef == VPS_COEF_CONST && C.degree >= 2 && C.degree <= 5 &&
         C.algorithm == VPS_ALG_COMBINED && C.patch_order == 0 && C.patches_per_block == 0;
}

int stream_min(const vps_context* c) {
  if (c->cfg.dim == 3 && c->cfg.degree == 5) return 1;  // the single-pass 3D tiles exceed the LDS at k = 5
  return c->cfg.stream_min_cells > 0 ? c->cfg.stream_min_cells : 32;
}

// 2D grid transfers: the row-streaming kernels on coarse levels of at least this many
// cells (vps_config.stream_min_cells when set, 256 otherwise)
int stream2_transfer_min(const vps_context* c) { return c->cfg.stream_min_cells > 0 ? c->cfg.stream_min_cells : 256; }

vps_dtype vdt(const vps_context* c) { return (vps_dtype)c->cfg.vcycle_dtype; }

// ---- level operations (dtype t) ----

hipError_t do_operator(vps_context* c, int l, const void* u, const void* b, void* out, vps_dtype t);

hipError_t do_smooth_color(vps_context* c, int l, void* u, const void* b, vps_dtype t, int color, int vlo = 0,
                           int vhi = 0) {
  const Level& L = c->lv[l];
  const int k = c->cfg.degree, d = c->cfg.dim, coef = c->cfg.coef;
  vps::PatchLaunch P{};
  P.u = u;
  P.b = b;
  P.rho = (coef == VPS_COEF_CONST) ? nullptr : (t == VPS_F64 ? (const void*)L.rho64 : (const void*)L.rho32);
  P.scal = L.scal;
  P.n1 = L.n1;
  P.ncell = L.ncell;
  P.color = color;
  P.coef = coef;
  P.pb = c->cfg.patches_per_block;  // 0: the launcher chooses
  P.order = c->cfg.patch_order;
  // automatic (sweeps measured per degree, precision and level size): a row of
  // patches per wave (degree 5: per workgroup of two waves) at degree 2 from 32
  // cells per direction, at degrees 3 to 5 from 64; otherwise pairs from 32 cells
  // except FP32 at degree 4 and at degree 5 (no pair kernel); one patch per wave
  // on smaller levels (too few groups to fill the chip)
  const int deg = c->cfg.degree;
  const bool row_auto = (deg == 2 && L.ncell >= 32) || (deg >= 3 && L.ncell >= 64);
  const bool pair_auto = L.ncell >= 32 && !(t == VPS_F32 && deg == 4) && deg <= 4;
  int ppw = c->cfg.patches_per_wave;
  if (ppw == 0) ppw = row_auto ? 3 : (pair_auto ? 2 : 1);
  P.ppw = (ppw == 3 ? row_kernel_applies(c->cfg) : pair_kernel_applies(c->cfg)) ? ppw : 1;
  P.row2 = c->cfg.wave_rows_2d;
  P.vlo = vlo;
  P.vhi = vhi;
  if (coef == VPS_COEF_CONST) {
    P.M[0] = L.Mfull.data();
    P.M[1] = nullptr;
    P.Kst[0] = L.Kfull.data();
    P.Kst[1] = nullptr;
  } else {
    P.M[0] = L.Mh[0].data();
    P.M[1] = L.Mh[1].data();
    P.Kst[0] = L.Kh[0].data();
    P.Kst[1] = L.Kh[1].data();
  }
  P.T1 = L.T1.data();
  P.lam = L.lam.data();
  P.Te = L.Te.empty() ? nullptr : L.Te.data();
  P.To = L.Te.empty() ? nullptr : L.To.data();
  P.lam_int = L.lam_int.empty() ? nullptr : L.lam_int.data();
  if (coef == VPS_COEF_CELL_EXACT) {
    // exact dense local solvers (the ceiling of any per-patch correction of the FDM inverse):
    // the global residual of the current iterate, then u_I += A_j(rho)^{-1} r_I on the color
    hipError_t e = do_operator(c, l, u, b, L.sep_r, t);
    if (e != hipSuccess) return e;
    return vps::launch_exact_apply((double*)u, (const double*)L.sep_r, L.binv, L.n1, L.ncell, color, c->stream);
  }
  if (c->cfg.algorithm == VPS_ALG_SEPARATED) {
    // Algorithm 3: global residual, then the local solves of the color's patches
    hipError_t e = do_operator(c, l, u, b, L.sep_r, t);
    if (e != hipSuccess) return e;
    return dispatch_tk(t, k, [&]<typename T, int K>() { return vps::launch_patch_solve<T, K>(P, L.sep_r, c->stream); });
  }
  if (!P.lam_int || !P.Te) P.pb = P.pb > 0 ? P.pb : -1;  // -1: generic kernel, automatic batch
  return dispatch_tkd(t, k, d, [&]<typename T, int K, int D>() { return vps::launch_patch_color<T, K, D>(P, c->stream); });
}

hipError_t do_smooth(vps_context* c, int l, void* u, const void* b, vps_dtype t, int sweeps, bool reverse) {
  const int nc = 1 << c->cfg.dim;
  const int N = c->lv[l].ncell, B = c->cfg.batch_layers;
  if (N < 2) return hipSuccess;
  if (B > 0 && N - 1 > 2 * B) {
    // Algorithm 5: slabs of B vertex layers, all colors of a slab before the next slab (levels with
    // more than 2B layers; the smaller ones fit the Infinity Cache whole and sweep whole colors)
    const int nb = (N - 2) / B + 1;
    for (int s = 0; s < sweeps; ++s)
      for (int i = 0; i < nb; ++i) {
        const int bi = reverse ? nb - 1 - i : i;
        for (int j = 0; j < nc; ++j) {
          hipError_t e = do_smooth_color(c, l, u, b, t, reverse ? nc - 1 - j : j, 1 + bi * B, std::min(N - 1, (bi + 1) * B));
          if (e != hipSuccess) return e;
        }
      }
    return hipSuccess;
  }
  for (int s = 0; s < sweeps; ++s)
    for (int i = 0; i < nc; ++i) {
      hipError_t e = do_smooth_color(c, l, u, b, t, reverse ? nc - 1 - i : i);
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

hipError_t do_operator(vps_context* c, int l, const void* u, const void* b, void* out, vps_dtype t) {
  const Level& L = c->lv[l];
  const int k = c->cfg.degree, d = c->cfg.dim;
  if (c->cfg.coef == VPS_COEF_CONST && d == 3 && L.ncell >= stream_min(c)) {
    vps::StreamLaunch S{u, b, out, L.n1, L.n1, L.ncell, L.sG0.data(), L.sG1.data(), L.sZ0.data(), L.sZ1.data()};
    return dispatch_tk(t, k, [&]<typename TT, int K>() { return vps::launch_stream_operator<TT, K>(S, c->stream); });
  }
  if (c->cfg.coef == VPS_COEF_CONST && d == 2 && L.ncell >= stream_min(c)) {
    vps::Stream2Launch S{u, b, out, L.n1, L.ncell, L.Mc.data(), L.Kc.data()};
    return dispatch_tk(t, k, [&]<typename TT, int K>() { return vps::launch_stream2_operator<TT, K>(S, c->stream); });
  }
  if (c->cfg.coef == VPS_COEF_CONST) {
    vps::TileLaunch T{};
    T.in = u;
    T.b = b;
    T.out = out;
    T.n1_in = L.n1;
    T.n1_out = L.n1;
    const int tc = vps::op_tc(k, d);
    T.tiles = (L.ncell + tc - 1) / tc;
    T.G0 = L.opM.data();
    T.G1 = L.opK.data();
    return dispatch_tkd(t, k, d, [&]<typename TT, int K, int D>() { return vps::launch_operator<TT, K, D>(T, c->stream); });
  }
  vps::VarOpLaunch V{};
  V.u = u;
  V.b = b;
  V.out = out;
  V.rho = (t == VPS_F64) ? (const void*)L.rho64 : (const void*)L.rho32;
  V.n1 = L.n1;
  V.ncell = L.ncell;
  V.Mc = L.Mc.data();
  V.Kc = L.Kc.data();
  return dispatch_tkd(t, k, d, [&]<typename TT, int K, int D>() { return vps::launch_operator_var<TT, K, D>(V, c->stream); });
}

hipError_t do_restrict(vps_context* c, int l, const void* rf, void* rc, vps_dtype t) {
  const int k = c->cfg.degree, d = c->cfg.dim;
  if (d == 3 && c->lv[l - 1].ncell >= stream_min(c)) {
    const Level& L = c->lv[l];
    vps::StreamLaunch S{rf, nullptr, rc, L.n1, c->lv[l - 1].n1, c->lv[l - 1].ncell, L.rG.data(), nullptr,
                        L.rZ.data(), nullptr};
    return dispatch_tk(t, k, [&]<typename TT, int K>() { return vps::launch_stream_restrict<TT, K>(S, c->stream); });
  }
  // 2D: the row-streaming restriction walks coarse cells one fine row at a time, which
  // pays from 256 coarse cells per direction and up to degree 4 (measured; below, and
  // at degree 5, the single-pass tiles are faster)
  if (d == 2 && k <= 4 && c->lv[l - 1].ncell >= stream2_transfer_min(c)) {
    const Level& L = c->lv[l];
    vps::Stream2Launch S{rf, nullptr, rc, 0, c->lv[l - 1].ncell, L.rG.data(), L.rZ.data()};
    return dispatch_tk(t, k, [&]<typename TT, int K>() { return vps::launch_stream2_restrict<TT, K>(S, c->stream); });
  }
  vps::TileLaunch T{};
  T.in = rf;
  T.out = rc;
  T.n1_in = c->lv[l].n1;
  T.n1_out = c->lv[l - 1].n1;
  const int tc = vps::restrict_tc(k, d);
  T.tiles = (c->lv[l - 1].ncell + tc - 1) / tc;
  T.G0 = c->lv[l].restrictG.data();
  return dispatch_tkd(t, k, d, [&]<typename TT, int K, int D>() { return vps::launch_restrict<TT, K, D>(T, c->stream); });
}

hipError_t do_prolong(vps_context* c, int l, const void* ec, void* uf, vps_dtype t) {
  const int k = c->cfg.degree, d = c->cfg.dim;
  if (d == 3 && c->lv[l - 1].ncell >= stream_min(c)) {
    const Level& L = c->lv[l];
    vps::StreamLaunch S{ec, nullptr, uf, c->lv[l - 1].n1, L.n1, c->lv[l - 1].ncell, L.pG.data(), nullptr,
                        L.pG.data(), nullptr};
    return dispatch_tk(t, k, [&]<typename TT, int K>() { return vps::launch_stream_prolong<TT, K>(S, c->stream); });
  }
  if (d == 2 && c->lv[l - 1].ncell >= stream2_transfer_min(c)) {  // 2D: from 256 coarse cells (measured)
    const Level& L = c->lv[l];
    vps::Stream2Launch S{ec, nullptr, uf, 0, c->lv[l - 1].ncell, L.pG.data(), nullptr};
    return dispatch_tk(t, k, [&]<typename TT, int K>() { return vps::launch_stream2_prolong<TT, K>(S, c->stream); });
  }
  vps::TileLaunch T{};
  T.in = ec;
  T.out = uf;
  T.n1_in = c->lv[l - 1].n1;
  T.n1_out = c->lv[l].n1;
  const int tc = vps::prolong_tc(k, d);
  T.tiles = (c->lv[l - 1].ncell + tc - 1) / tc;
  T.G0 = c->lv[l].prolongG.data();
  return dispatch_tkd(t, k, d, [&]<typename TT, int K, int D>() { return vps::launch_prolong<TT, K, D>(T, c->stream); });
}

hipError_t do_coarse(vps_context* c, const void* b, void* x, vps_dtype t) {
  const int d = c->cfg.dim;
  const int ti = (t == VPS_F64) ? 0 : 1;
  if (c->cfg.coef == VPS_COEF_CONST) {
    vps::CoarseFdmLaunch C{b, x, c->cn0, c->cT0[ti], c->clam0[ti]};
    if (t == VPS_F64) return d == 3 ? vps::launch_coarse_fdm<double, 3>(C, c->stream) : vps::launch_coarse_fdm<double, 2>(C, c->stream);
    return d == 3 ? vps::launch_coarse_fdm<float, 3>(C, c->stream) : vps::launch_coarse_fdm<float, 2>(C, c->stream);
  }
  if (t == VPS_F64)
    return vps::launch_coarse_dense<double>(c->cAinv[0], c->cfree, c->cnfree, b, x, c->lv[0].nodes, c->stream);
  return vps::launch_coarse_dense<float>(c->cAinv[1], c->cfree, c->cnfree, b, x, c->lv[0].nodes, c->stream);
}

hipError_t vcycle_level(vps_context* c, int l, const void* b, void* u) {
  const vps_dtype t = vdt(c);
  hipError_t e;
  if (l == 0) {
    const int i0 = tbegin(c, PH_COARSE, 0);
    e = do_coarse(c, b, u, t);
    tend(c, i0);
    return e;
  }
  Level& L = c->lv[l];
  int ti = tbegin(c, PH_SMOOTH, l, c->cfg.pre_sweeps);
  if (t == VPS_F64) e = vps::launch_fill<double>(u, 0.0, L.nodes, c->stream);
  else e = vps::launch_fill<float>(u, 0.0, L.nodes, c->stream);
  if (e != hipSuccess) return e;
  if ((e = do_smooth(c, l, u, b, t, c->cfg.pre_sweeps, false)) != hipSuccess) return e;
  tend(c, ti);
  ti = tbegin(c, PH_RESIDUAL, l);
  if ((e = do_operator(c, l, u, b, L.r, t)) != hipSuccess) return e;
  tend(c, ti);
  ti = tbegin(c, PH_RESTRICT, l);
  if ((e = do_restrict(c, l, L.r, c->lv[l - 1].b, t)) != hipSuccess) return e;
  tend(c, ti);
  if ((e = vcycle_level(c, l - 1, c->lv[l - 1].b, c->lv[l - 1].u)) != hipSuccess) return e;
  ti = tbegin(c, PH_PROLONG, l);
  if ((e = do_prolong(c, l, c->lv[l - 1].u, u, t)) != hipSuccess) return e;
  tend(c, ti);
  ti = tbegin(c, PH_SMOOTH, l, c->cfg.post_sweeps);
  e = do_smooth(c, l, u, b, t, c->cfg.post_sweeps, true);
  tend(c, ti);
  return e;
}

void drop_graphs(vps_context* c) {
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  c->graphs.clear();
}

// The finest-level V-cycle from b into u.  With vps_config.vcycle_graph, once
// per (b, u) pair its launches are captured on a private stream into a HIP
// graph, which later calls replay on the context stream: one launch instead
// of a few hundred.  Kernel by kernel otherwise, while the phase timer runs
// (its events sit between the launches), or after a failed capture.
hipError_t finest_vcycle(vps_context* c, const void* b, void* u) {
  const int L = (int)c->lv.size() - 1;
  if (!c->cfg.vcycle_graph || c->timer.on || c->graphs_failed) return vcycle_level(c, L, b, u);
  for (const auto& g : c->graphs)
    if (g.b == b && g.u == u) return hipGraphLaunch(g.exec, c->stream);
  hipError_t e = hipSuccess;
  if (!c->capture_stream && (e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking)) != hipSuccess) {
    c->graphs_failed = true;
    return vcycle_level(c, L, b, u);
  }
  const hipStream_t user = c->stream;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  e = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    c->stream = c->capture_stream;
    const hipError_t ev = vcycle_level(c, L, b, u);
    c->stream = user;
    e = hipStreamEndCapture(c->capture_stream, &graph);
    if (ev != hipSuccess) e = ev;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    c->graphs_failed = true;
    (void)hipGetLastError();
    return vcycle_level(c, L, b, u);
  }
  if (c->graphs.size() >= 4) {  // keep a few: the solvers use one or two pairs
    (void)hipGraphExecDestroy(c->graphs.front().exec);
    c->graphs.erase(c->graphs.begin());
  }
  c->graphs.push_back({b, u, exec});
  return hipGraphLaunch(exec, c->stream);
}

hipError_t do_vcycle(vps_context* c, const double* r, double* z) {
  const int L = (int)c->lv.size() - 1;
  if (c->timer.on) c->timer.tot.vcycles += 1;
  if (vdt(c) == VPS_F64) return finest_vcycle(c, r, z);
  Level& F = c->lv[L];
  int ti = tbegin(c, PH_CG_VEC, L);
  hipError_t e = vps::launch_cast<double, float>(r, F.b, F.nodes, c->stream);
  if (e != hipSuccess) return e;
  tend(c, ti);
  if ((e = finest_vcycle(c, F.b, F.u)) != hipSuccess) return e;
  ti = tbegin(c, PH_CG_VEC, L);
  e = vps::launch_cast<float, double>(F.u, z, F.nodes, c->stream);
  tend(c, ti);
  return e;
}

vps_status need_coarse(vps_context* c) {
  if (!c->coarse_ok)
    return fail(c, VPS_E_UNSUPPORTED,
                "no coarse solver for this coarsest grid (rho = 1: at most 15 free nodes per direction in 3D, "
                "63 in 2D; cell coefficient: at most 4096 free nodes)");
  return VPS_OK;
}

vps_status need_coef(vps_context* c) {
  if (c->cfg.coef != VPS_COEF_CONST && !c->coef_set)
    return fail(c, VPS_E_STATE, "the cell coefficient has not been set (vps_set_coefficient)");
  return VPS_OK;
}

// host reads of device dot products
vps_status dots(vps_context* c, const double* x, const double* y, const double* x2, const double* y2, size_t n,
                double* out) {
  int nblk = 0;
  VPS_HIP(c, vps::launch_dot_partial(x, y, x2, y2, n, c->partial, &nblk, c->stream));
  const int nd = x2 ? 2 : 1;
  VPS_HIP(c, vps::launch_dot_final(c->partial, nblk, nd, c->dscal, c->stream));
  VPS_HIP(c, hipMemcpyAsync(c->hscal, c->dscal, nd * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  VPS_HIP(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < nd; ++i) out[i] = c->hscal[i];
  return VPS_OK;
}

// One FP32 V-cycle on the finest level: F.b holds the residual in FP32, the
// correction is left in F.u (FP32).
hipError_t vcycle_f32_resident(vps_context* c) {
  const int L = (int)c->lv.size() - 1;
  if (c->timer.on) c->timer.tot.vcycles += 1;
  return finest_vcycle(c, c->lv[L].b, c->lv[L].u);
}

vps_status dots_z32(vps_context* c, const double* r, const float* z, const double* q, size_t n, double* out) {
  int nblk = 0;
  VPS_HIP(c, vps::launch_dot_z32(r, z, q, n, c->partial, &nblk, c->stream));
  const int nd = q ? 2 : 1;
  VPS_HIP(c, vps::launch_dot_final(c->partial, nblk, nd, c->dscal, c->stream));
  VPS_HIP(c, hipMemcpyAsync(c->hscal, c->dscal, nd * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  VPS_HIP(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < nd; ++i) out[i] = c->hscal[i];
  return VPS_OK;
}

vps_status ensure_cg(vps_context* c) {
  if (c->cg_r) return VPS_OK;
  const size_t n = c->lv.back().nodes * sizeof(double);
  VPS_HIP(c, hipMalloc(&c->cg_r, n));
  VPS_HIP(c, hipMalloc(&c->cg_p, n));
  VPS_HIP(c, hipMalloc(&c->cg_q, n));
  VPS_HIP(c, hipMalloc(&c->cg_z, n));
  return VPS_OK;
}

void free_all(vps_context* c) {
  drop_graphs(c);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  c->capture_stream = nullptr;
  for (Level& L : c->lv) {
    hipFree(L.u);
    hipFree(L.b);
    hipFree(L.r);
    hipFree(L.sep_r);
    hipFree(L.rho64);
    hipFree(L.rho32);
    hipFree(L.scal);
    hipFree(L.binv);
  }
  for (int i = 0; i < 2; ++i) {
    hipFree(c->cT0[i]);
    hipFree(c->clam0[i]);
    hipFree(c->cAinv[i]);
  }
  hipFree(c->cfree);
  hipFree(c->cg_r);
  hipFree(c->cg_p);
  hipFree(c->cg_q);
  hipFree(c->cg_z);
  hipFree(c->partial);
  hipFree(c->dscal);
  if (c->hscal) hipHostFree(c->hscal);
  if (c->ev0) hipEventDestroy(c->ev0);
  if (c->ev1) hipEventDestroy(c->ev1);
  for (hipEvent_t e : c->timer.pool) hipEventDestroy(e);
  vps::mlp_free(&c->mlp);
}

}  // namespace

extern "C" {

const char* vps_status_string(vps_status s) {
  const int i = -(int)s;
  if (i < 0 || i >= (int)(sizeof(kStatusText) / sizeof(kStatusText[0]))) return "unknown status";
  return kStatusText[i];
}

const char* vps_last_error(const vps_context* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

vps_status vps_create(const vps_config* cfg, void* hip_stream, vps_context** out) {
  if (!cfg || !out) return VPS_E_ARG;
  *out = nullptr;
  const vps_config& C = *cfg;
  if (C.dim != 2 && C.dim != 3) return VPS_E_UNSUPPORTED;
  if (C.degree < 1 || C.degree > 5) return VPS_E_UNSUPPORTED;
  if (C.n_levels < 1 || C.n_cells < 2) return VPS_E_UNSUPPORTED;
  if (C.n_levels > VPS_MAX_LEVELS || C.n_cells % (1 << (C.n_levels - 1)) != 0) return VPS_E_UNSUPPORTED;
  const int n0 = C.n_cells >> (C.n_levels - 1);
  if (n0 < 2) return VPS_E_UNSUPPORTED;
  if (C.pre_sweeps < 0 || C.post_sweeps < 0) return VPS_E_ARG;
  if (C.vcycle_dtype != VPS_F64 && C.vcycle_dtype != VPS_F32) return VPS_E_ARG;
  if (C.coef < VPS_COEF_CONST || C.coef > VPS_COEF_CELL_EXACT) return VPS_E_ARG;
  // dense exact local solvers: Q2 in 3D, FP64, whole colors (each color step: the global
  // residual, then the dense patch solves)
  if (C.coef == VPS_COEF_CELL_EXACT &&
      (C.dim != 3 || C.degree != 2 || C.vcycle_dtype != VPS_F64 || C.algorithm != VPS_ALG_COMBINED ||
       C.batch_layers != 0 || C.patches_per_block != 0))
    return VPS_E_UNSUPPORTED;
  if (C.patches_per_block != 0 && !vps::valid_patches_per_block(C.patches_per_block)) return VPS_E_UNSUPPORTED;
  if (C.patches_per_block != 0 && C.dim >= 2 && C.dim <= 3 && C.degree >= 1 && C.degree <= 5 &&
      C.coef >= VPS_COEF_CONST && C.coef <= VPS_COEF_CELL_EXACT &&
      !vps::patches_per_block_fits(C.degree, C.dim, C.coef, C.patches_per_block, C.vcycle_dtype == VPS_F64))
    return VPS_E_UNSUPPORTED;  // that batch of patches exceeds the workgroup LDS
  if (C.stream_min_cells < 0) return VPS_E_ARG;
  if (C.algorithm != VPS_ALG_COMBINED && C.algorithm != VPS_ALG_SEPARATED) return VPS_E_ARG;
  if (C.patch_order < 0 || C.patch_order > 3) return VPS_E_ARG;
  if (C.batch_layers < 0) return VPS_E_ARG;
  if (C.batch_layers > 0 && C.algorithm != VPS_ALG_COMBINED) return VPS_E_UNSUPPORTED;
  if (C.patches_per_wave < 0 || C.patches_per_wave > 3) return VPS_E_ARG;
  if (C.patches_per_wave == 2 && !pair_kernel_applies(C)) return VPS_E_UNSUPPORTED;
  if (C.patches_per_wave == 3 && !row_kernel_applies(C)) return VPS_E_UNSUPPORTED;
  if (C.vcycle_graph != 0 && C.vcycle_graph != 1) return VPS_E_ARG;
  if (C.wave_rows_2d < 0 || C.wave_rows_2d > 2) return VPS_E_ARG;
  if (C.wave_rows_2d == 1 && (C.dim != 2 || C.coef != VPS_COEF_CONST || C.degree < 2 || C.patches_per_block != 0))
    return VPS_E_UNSUPPORTED;
  if (C.algorithm == VPS_ALG_SEPARATED && (C.dim != 3 || C.coef != VPS_COEF_CONST || C.degree < 2 || C.degree > 4))
    return VPS_E_UNSUPPORTED;
  // every node index must fit in int on the kernels' inner indexing
  const double nodes = std::pow((double)(C.degree * C.n_cells + 1), C.dim);
  if (nodes > 2.0e9) return VPS_E_UNSUPPORTED;
  // the 3D constant-coefficient patch kernels (degree 2..4) address a level vector of the
  // V-cycle dtype with 32-bit byte offsets
  const double vbytes = nodes * (C.vcycle_dtype == VPS_F64 ? 8.0 : 4.0);
  if (C.dim == 3 && C.coef == VPS_COEF_CONST && C.degree >= 2 && C.degree <= 4 && vbytes >= 4294967296.0)
    return VPS_E_UNSUPPORTED;

  // the static work memory of vps_mlp_backward_noalloc: its device address, once per GPU
  if (hipError_t e = vps::mlp_scratch_setup(); e != hipSuccess) {
    g_create_error = std::string("vps_create: hipGetSymbolAddress of the static work memory: ") + hipGetErrorString(e);
    return VPS_E_HIP;
  }
  vps_context* c = new vps_context();
  c->cfg = C;
  c->stream = (hipStream_t)hip_stream;
  const vps_dtype t = (vps_dtype)C.vcycle_dtype;
  c->lv.resize(C.n_levels);
  c->fallback.assign(C.n_levels, 0);
  for (int l = 0; l < C.n_levels; ++l) build_level(c->lv[l], C.degree, C.dim, n0 << l);

  hipError_t last = hipSuccess;
  const char* what = "";
  auto bail = [&](vps_status s) {
    g_create_error = std::string("vps_create: ") + what + (last != hipSuccess ? std::string(": ") + hipGetErrorString(last) : "");
    free_all(c);
    delete c;
    return s;
  };
  auto chk = [&](hipError_t e, const char* w) {
    last = e;
    what = w;
    return e != hipSuccess;
  };
  for (Level& L : c->lv) {
    if (chk(hipMalloc(&L.u, L.nodes * esize(t)), "hipMalloc")) return bail(VPS_E_NOMEM);
    if (chk(hipMalloc(&L.b, L.nodes * esize(t)), "hipMalloc")) return bail(VPS_E_NOMEM);
    if (chk(hipMalloc(&L.r, L.nodes * esize(t)), "hipMalloc")) return bail(VPS_E_NOMEM);
    if (C.algorithm == VPS_ALG_SEPARATED && chk(hipMalloc(&L.sep_r, L.nodes * sizeof(double)), "hipMalloc"))
      return bail(VPS_E_NOMEM);
    if (C.coef != VPS_COEF_CONST) {
      size_t cells = 1;
      for (int e = 0; e < C.dim; ++e) cells *= (size_t)L.ncell;
      if (chk(hipMalloc(&L.rho64, cells * sizeof(double)), "hipMalloc")) return bail(VPS_E_NOMEM);
      if (chk(hipMalloc(&L.rho32, cells * sizeof(float)), "hipMalloc")) return bail(VPS_E_NOMEM);
    }
    if (C.coef == VPS_COEF_CELL_EXACT && L.npatch > 0) {
      if (chk(hipMalloc(&L.binv, (size_t)L.npatch * 27 * 27 * sizeof(double)), "hipMalloc")) return bail(VPS_E_NOMEM);
      if (chk(hipMalloc(&L.sep_r, L.nodes * sizeof(double)), "hipMalloc")) return bail(VPS_E_NOMEM);
    }
    if (C.coef == VPS_COEF_CELL_LEARNED) {
      const size_t n = (size_t)L.npatch * ipow(2 * C.degree - 1, C.dim);
      if (n > 0) {
        if (chk(hipMalloc(&L.scal, n * sizeof(float)), "hipMalloc")) return bail(VPS_E_NOMEM);
        if (chk(vps::launch_fill<float>(L.scal, 1.0, n, c->stream), "fill")) return bail(VPS_E_HIP);
      }
    }
  }
  if (C.coef == VPS_COEF_CONST && C.degree * n0 - 1 <= vps::coarse_fdm_max_n0(C.dim)) {
    // fast diagonalisation of the whole coarse grid (Kronecker sum of 1D matrices)
    const Level& L0 = c->lv[0];
    const int k = C.degree;
    Mat M, K;
    vps::assemble_1d(k, L0.ncell, L0.h, &M, &K);
    const int nn = k * L0.ncell + 1, m = nn - 2;
    Mat Mi(m * m), Ki(m * m), T0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        Mi[i * m + j] = M[(i + 1) * nn + j + 1];
        Ki[i * m + j] = K[(i + 1) * nn + j + 1];
      }
    std::vector<double> lam0;
    vps::gen_eig(m, Mi, Ki, &T0, &lam0);
    c->cn0 = m;
    if (chk(upload<double>(T0, &c->cT0[0], c->stream), "upload")) return bail(VPS_E_HIP);
    if (chk(upload<double>(lam0, &c->clam0[0], c->stream), "upload")) return bail(VPS_E_HIP);
    if (chk(upload<float>(T0, &c->cT0[1], c->stream), "upload")) return bail(VPS_E_HIP);
    if (chk(upload<float>(lam0, &c->clam0[1], c->stream), "upload")) return bail(VPS_E_HIP);
    c->coarse_ok = true;
  }
  if (chk(hipMalloc(&c->partial, 2 * vps::kDotBlocks * sizeof(double)), "hipMalloc")) return bail(VPS_E_NOMEM);
  if (chk(hipMalloc(&c->dscal, 4 * sizeof(double)), "hipMalloc")) return bail(VPS_E_NOMEM);
  if (chk(hipHostMalloc(&c->hscal, 4 * sizeof(double), 0), "hipHostMalloc")) return bail(VPS_E_NOMEM);
  if (chk(hipEventCreate(&c->ev0), "hipEventCreate") || chk(hipEventCreate(&c->ev1), "hipEventCreate")) return bail(VPS_E_HIP);
  if (chk(hipStreamSynchronize(c->stream), "hipStreamSynchronize")) return bail(VPS_E_HIP);
  *out = c;
  return VPS_OK;
}

vps_status vps_destroy(vps_context* ctx) {
  if (!ctx) return VPS_OK;
  hipStreamSynchronize(ctx->stream);
  free_all(ctx);
  delete ctx;
  return VPS_OK;
}

vps_status vps_set_stream(vps_context* ctx, void* hip_stream) {
  if (!ctx) return VPS_E_ARG;
  ctx->stream = (hipStream_t)hip_stream;
  return VPS_OK;
}

size_t vps_level_nodes(const vps_context* ctx, int level) { return level_ok(ctx, level) ? ctx->lv[level].nodes : 0; }

int vps_level_cells(const vps_context* ctx, int level) { return level_ok(ctx, level) ? ctx->lv[level].ncell : 0; }

long long vps_level_patches(const vps_context* ctx, int level) {
  return level_ok(ctx, level) ? ctx->lv[level].npatch : 0;
}

vps_status vps_set_coefficient(vps_context* c, const double* rho) {
  if (!c || !rho) return fail(c, VPS_E_ARG, "null argument");
  if (c->cfg.coef == VPS_COEF_CONST) return fail(c, VPS_E_STATE, "context was created with coef = VPS_COEF_CONST");
  drop_graphs(c);  // the coarse solver's buffers may be replaced
  const int d = c->cfg.dim, k = c->cfg.degree;
  const int L = (int)c->lv.size() - 1;
  auto cells = [&](int l) {
    size_t n = 1;
    for (int e = 0; e < d; ++e) n *= (size_t)c->lv[l].ncell;
    return n;
  };
  VPS_HIP(c, hipMemcpyAsync(c->lv[L].rho64, rho, cells(L) * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  for (int l = L - 1; l >= 0; --l)
    VPS_HIP(c, vps::launch_coarsen_rho(c->lv[l + 1].rho64, c->lv[l].rho64, c->lv[l].ncell, d, c->stream));
  for (int l = 0; l <= L; ++l)
    VPS_HIP(c, (vps::launch_cast<double, float>(c->lv[l].rho64, c->lv[l].rho32, cells(l), c->stream)));
  if (c->cfg.coef == VPS_COEF_CELL_EXACT)
    for (int l = 0; l <= L; ++l)
      if (c->lv[l].binv)
        VPS_HIP(c, vps::launch_exact_inverses(c->lv[l].rho64, c->lv[l].ncell, c->lv[l].Mh, c->lv[l].Kh, c->lv[l].binv,
                                              c->stream));
  // dense coarse operator on the free nodes, FP64 on the host
  const Level& L0 = c->lv[0];
  std::vector<double> rho0(cells(0));
  VPS_HIP(c, hipMemcpyAsync(rho0.data(), L0.rho64, rho0.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  VPS_HIP(c, hipStreamSynchronize(c->stream));
  for (double v : rho0)
    if (!(v > 0.0) || !std::isfinite(v)) return fail(c, VPS_E_ARG, "coefficient must be positive and finite");
  const int n1 = L0.n1, nf1 = n1 - 2;
  const int nfree = ipow(nf1, d);
  c->coef_set = true;
  if (nfree > kMaxDenseCoarse) {  // no coarse solver; smoother and operator still usable
    c->coarse_ok = false;
    return VPS_OK;
  }
  Mat A((size_t)nfree * nfree, 0.0);
  const int m1 = k + 1, mloc = ipow(m1, d);
  std::vector<int> gid(mloc);
  for (size_t cell = 0; cell < rho0.size(); ++cell) {
    int cc[3] = {(int)(cell % L0.ncell), (int)((cell / L0.ncell) % L0.ncell),
                 d == 3 ? (int)(cell / ((size_t)L0.ncell * L0.ncell)) : 0};
    for (int a = 0; a < mloc; ++a) {
      int id = 0, stride = 1;
      bool fr = true;
      int rem = a;
      for (int e = 0; e < d; ++e) {
        const int g = cc[e] * k + rem % m1;
        rem /= m1;
        if (g == 0 || g == n1 - 1) fr = false;
        id += (g - 1) * stride;
        stride *= nf1;
      }
      gid[a] = fr ? id : -1;
    }
    for (int a = 0; a < mloc; ++a) {
      if (gid[a] < 0) continue;
      for (int bb = 0; bb < mloc; ++bb) {
        if (gid[bb] < 0) continue;
        double v = 0.0;
        for (int e = 0; e < d; ++e) {
          double prod = 1.0;
          int ra = a, rb = bb;
          for (int ep = 0; ep < d; ++ep) {
            const int ia = ra % m1, ib = rb % m1;
            ra /= m1;
            rb /= m1;
            prod *= (ep == e) ? L0.Kc[ia * m1 + ib] : L0.Mc[ia * m1 + ib];
          }
          v += prod;
        }
        A[(size_t)gid[a] * nfree + gid[bb]] += rho0[cell] * v;
      }
    }
  }
  if (!vps::spd_inverse(nfree, &A)) return fail(c, VPS_E_NONFINITE, "coarse operator is not SPD");
  std::vector<int> fidx_i(nfree);
  for (int i = 0; i < nfree; ++i) {
    int rem = i, g = 0, stride = 1;
    for (int e = 0; e < d; ++e) {
      g += (rem % nf1 + 1) * stride;
      rem /= nf1;
      stride *= n1;
    }
    fidx_i[i] = g;
  }
  for (int i = 0; i < 2; ++i) {
    hipFree(c->cAinv[i]);
    c->cAinv[i] = nullptr;
  }
  hipFree(c->cfree);
  c->cfree = nullptr;
  VPS_HIP(c, upload<double>(A, &c->cAinv[0], c->stream));
  VPS_HIP(c, upload<float>(A, &c->cAinv[1], c->stream));
  VPS_HIP(c, hipMalloc(&c->cfree, nfree * sizeof(int)));
  VPS_HIP(c, hipMemcpyAsync(c->cfree, fidx_i.data(), nfree * sizeof(int), hipMemcpyHostToDevice, c->stream));
  VPS_HIP(c, hipStreamSynchronize(c->stream));
  c->cnfree = nfree;
  c->coarse_ok = true;
  return VPS_OK;
}

vps_status vps_set_patch_scaling(vps_context* c, int level, const float* cdev) {
  if (!c) return VPS_E_ARG;
  if (!level_ok(c, level)) return fail(c, VPS_E_ARG, "invalid level");
  if (c->cfg.coef != VPS_COEF_CELL_LEARNED) return fail(c, VPS_E_STATE, "context was not created with learned scaling");
  drop_graphs(c);
  Level& L = c->lv[level];
  const size_t n = (size_t)L.npatch * ipow(2 * c->cfg.degree - 1, c->cfg.dim);
  if (n == 0) return VPS_OK;
  if (cdev) VPS_HIP(c, hipMemcpyAsync(L.scal, cdev, n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  else VPS_HIP(c, vps::launch_fill<float>(L.scal, 1.0, n, c->stream));
  return VPS_OK;
}

vps_status vps_apply(vps_context* c, int level, const void* u, void* Au, vps_dtype t) {
  if (!c || !u || !Au) return fail(c, VPS_E_ARG, "null argument");
  if (!level_ok(c, level)) return fail(c, VPS_E_ARG, "invalid level");
  if (t != VPS_F64 && t != VPS_F32) return fail(c, VPS_E_ARG, "invalid dtype");
  if (vps_status s = need_coef(c)) return s;
  VPS_HIP(c, do_operator(c, level, u, nullptr, Au, t));
  return VPS_OK;
}

vps_status vps_residual(vps_context* c, int level, const void* b, const void* u, void* r, vps_dtype t) {
  if (!c || !u || !b || !r) return fail(c, VPS_E_ARG, "null argument");
  if (!level_ok(c, level)) return fail(c, VPS_E_ARG, "invalid level");
  if (t != VPS_F64 && t != VPS_F32) return fail(c, VPS_E_ARG, "invalid dtype");
  if (vps_status s = need_coef(c)) return s;
  VPS_HIP(c, do_operator(c, level, u, b, r, t));
  return VPS_OK;
}

vps_status vps_restrict(vps_context* c, int fine_level, const void* rf, void* rc, vps_dtype t) {
  if (!c || !rf || !rc) return fail(c, VPS_E_ARG, "null argument");
  if (!level_ok(c, fine_level) || fine_level == 0) return fail(c, VPS_E_ARG, "invalid fine level");
  if (t != VPS_F64 && t != VPS_F32) return fail(c, VPS_E_ARG, "invalid dtype");
  VPS_HIP(c, do_restrict(c, fine_level, rf, rc, t));
  return VPS_OK;
}

vps_status vps_prolongate_add(vps_context* c, int fine_level, const void* ec, void* uf, vps_dtype t) {
  if (!c || !ec || !uf) return fail(c, VPS_E_ARG, "null argument");
  if (!level_ok(c, fine_level) || fine_level == 0) return fail(c, VPS_E_ARG, "invalid fine level");
  if (t != VPS_F64 && t != VPS_F32) return fail(c, VPS_E_ARG, "invalid dtype");
  VPS_HIP(c, do_prolong(c, fine_level, ec, uf, t));
  return VPS_OK;
}

vps_status vps_coarse_solve(vps_context* c, const void* b, void* x, vps_dtype t) {
  if (!c || !b || !x) return fail(c, VPS_E_ARG, "null argument");
  if (t != VPS_F64 && t != VPS_F32) return fail(c, VPS_E_ARG, "invalid dtype");
  if (vps_status s = need_coef(c)) return s;
  if (vps_status s = need_coarse(c)) return s;
  VPS_HIP(c, do_coarse(c, b, x, t));
  return VPS_OK;
}

vps_status vps_smooth_color(vps_context* c, int level, void* u, const void* b, vps_dtype t, int color) {
  if (!c || !u || !b) return fail(c, VPS_E_ARG, "null argument");
  if (!level_ok(c, level)) return fail(c, VPS_E_ARG, "invalid level");
  if (t != VPS_F64 && t != VPS_F32) return fail(c, VPS_E_ARG, "invalid dtype");
  if (color < 0 || color >= (1 << c->cfg.dim)) return fail(c, VPS_E_ARG, "invalid color");
  if (vps_status s = need_coef(c)) return s;
  if (c->lv[level].ncell < 2) return VPS_OK;
  VPS_HIP(c, do_smooth_color(c, level, u, b, t, color));
  return VPS_OK;
}

vps_status vps_smooth(vps_context* c, int level, void* u, const void* b, vps_dtype t, int sweeps, int reverse) {
  if (!c || !u || !b) return fail(c, VPS_E_ARG, "null argument");
  if (!level_ok(c, level)) return fail(c, VPS_E_ARG, "invalid level");
  if (t != VPS_F64 && t != VPS_F32) return fail(c, VPS_E_ARG, "invalid dtype");
  if (sweeps < 0) return fail(c, VPS_E_ARG, "negative sweeps");
  if (vps_status s = need_coef(c)) return s;
  const int ti = tbegin(c, PH_SMOOTH, level, sweeps);
  VPS_HIP(c, do_smooth(c, level, u, b, t, sweeps, reverse != 0));
  tend(c, ti);
  return VPS_OK;
}

vps_status vps_vcycle(vps_context* c, const double* r, double* z) {
  if (!c || !r || !z) return fail(c, VPS_E_ARG, "null argument");
  if (vps_status s = need_coef(c)) return s;
  if (vps_status s = need_coarse(c)) return s;
  VPS_HIP(c, do_vcycle(c, r, z));
  return VPS_OK;
}

// Preconditioned CG in FP64 (Section 4).  With an FP32 V-cycle the
// preconditioner is not exactly symmetric, so the flexible form is used:
// beta = (z_new, r_new - r_old) / (z_old, r_old) with r_new - r_old = -alpha q.
// FP32 V-cycle: the CG update writes the FP32 residual the V-cycle reads, and
// the FP32 correction is consumed directly by the dot products and the update
// of the search direction (no FP64 copy of it).
vps_status vps_solve(vps_context* c, const double* b, double* x, double rtol, int maxit, vps_solve_info* info) {
  if (!c || !b || !x) return fail(c, VPS_E_ARG, "null argument");
  if (!(rtol > 0.0) || maxit < 0) return fail(c, VPS_E_ARG, "rtol must be > 0 and maxit >= 0");
  if (vps_status s = need_coef(c)) return s;
  if (vps_status s = need_coarse(c)) return s;
  if (vps_status s = ensure_cg(c)) return s;
  const int L = (int)c->lv.size() - 1;
  const size_t n = c->lv[L].nodes;
  const bool mixed = vdt(c) == VPS_F32;
  double *r = c->cg_r, *p = c->cg_p, *q = c->cg_q, *z = c->cg_z;
  float* r32 = mixed ? (float*)c->lv[L].b : nullptr;
  const float* z32 = mixed ? (const float*)c->lv[L].u : nullptr;
  vps_solve_info inf{};
  for (long long f : c->fallback) inf.fallback_patches += f;
  VPS_HIP(c, hipEventRecord(c->ev0, c->stream));
  double s2[2];
  if (vps_status st = dots(c, b, b, nullptr, nullptr, n, s2)) return st;
  const double bn = std::sqrt(s2[0]);
  if (!std::isfinite(bn)) return fail(c, VPS_E_NONFINITE, "right-hand side is not finite");
  vps_status result = VPS_E_NOT_CONVERGED;
  bool x_set = false;  // x is written by the first update (x_0 = 0)
  double true_rn = -1.0;  // ||b - A x|| of the final x once computed
  if (bn == 0.0) {
    result = VPS_OK;
  } else if (maxit > 0) {
    // z_0 = M b, p_0 = z_0
    double rz;
    int ti;
    if (mixed) {
      ti = tbegin(c, PH_CG_VEC, L);
      VPS_HIP(c, (vps::launch_cast<double, float>(b, r32, n, c->stream)));
      tend(c, ti);
      VPS_HIP(c, vcycle_f32_resident(c));
      ti = tbegin(c, PH_CG_VEC, L);
      if (vps_status st = dots_z32(c, b, z32, nullptr, n, s2)) return st;
      VPS_HIP(c, (vps::launch_cast<float, double>(z32, p, n, c->stream)));
      tend(c, ti);
    } else {
      VPS_HIP(c, do_vcycle(c, b, z));
      if (vps_status st = dots(c, b, z, nullptr, nullptr, n, s2)) return st;
      std::swap(p, z);  // p_0 = z_0 without a copy; z is overwritten by the next V-cycle
    }
    rz = s2[0];
    int it = 0;
    while (it < maxit) {
      ++it;
      ti = tbegin(c, PH_CG_OP, L);
      VPS_HIP(c, do_operator(c, L, p, nullptr, q, VPS_F64));
      tend(c, ti);
      ti = tbegin(c, PH_CG_VEC, L);
      if (vps_status st = dots(c, p, q, nullptr, nullptr, n, s2)) return st;
      const double pq = s2[0];
      const double alpha = rz / pq;
      if (!std::isfinite(alpha) || !(pq > 0.0)) {
        inf.iterations = it;
        result = fail(c, VPS_E_NONFINITE, "CG breakdown: (p, A p) is not positive and finite");
        break;
      }
      int nblk = 0;
      VPS_HIP(c, vps::launch_cg_update(alpha, p, q, x, x_set ? r : b, r, r32, !x_set, n, c->partial, &nblk,
                                       c->stream));
      x_set = true;
      VPS_HIP(c, vps::launch_dot_final(c->partial, nblk, 1, c->dscal, c->stream));
      VPS_HIP(c, hipMemcpyAsync(c->hscal, c->dscal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
      VPS_HIP(c, hipStreamSynchronize(c->stream));
      tend(c, ti);
      double rn = std::sqrt(c->hscal[0]);
      inf.iterations = it;
      if (!std::isfinite(rn)) {
        result = fail(c, VPS_E_NONFINITE, "residual norm is not finite");
        break;
      }
      bool restarted = false;
      if (rn <= rtol * bn) {
        // confirm with the true residual
        VPS_HIP(c, do_operator(c, L, x, b, r, VPS_F64));
        if (vps_status st = dots(c, r, r, nullptr, nullptr, n, s2)) return st;
        rn = std::sqrt(s2[0]);
        if (rn <= rtol * bn) {
          result = VPS_OK;
          true_rn = rn;
          break;
        }
        restarted = true;
        if (mixed) VPS_HIP(c, (vps::launch_cast<double, float>(r, r32, n, c->stream)));
      }
      double rzn, zq = 0.0;
      if (mixed) {
        VPS_HIP(c, vcycle_f32_resident(c));
        ti = tbegin(c, PH_CG_VEC, L);
        if (vps_status st = dots_z32(c, r, z32, restarted ? nullptr : q, n, s2)) return st;
      } else {
        VPS_HIP(c, do_vcycle(c, r, z));
        ti = tbegin(c, PH_CG_VEC, L);
        if (vps_status st = dots(c, r, z, nullptr, nullptr, n, s2)) return st;
      }
      rzn = s2[0];
      if (mixed && !restarted) zq = s2[1];
      const double beta = (mixed && !restarted) ? (-alpha * zq) / rz : rzn / rz;
      rz = rzn;
      if (!std::isfinite(beta)) {
        result = fail(c, VPS_E_NONFINITE, "CG breakdown: beta is not finite");
        break;
      }
      if (mixed) VPS_HIP(c, vps::launch_xpay_z32(z32, beta, p, n, c->stream));
      else VPS_HIP(c, vps::launch_xpay(z, beta, p, n, c->stream));
      tend(c, ti);
    }
  }
  if (!x_set) VPS_HIP(c, vps::launch_fill<double>(x, 0.0, n, c->stream));
  // final true residual (already at hand when the convergence test computed it for this x)
  if (true_rn < 0.0) {
    VPS_HIP(c, do_operator(c, L, x, b, q, VPS_F64));
    if (vps_status st = dots(c, q, q, nullptr, nullptr, n, s2)) return st;
    true_rn = std::sqrt(s2[0]);
  }
  VPS_HIP(c, hipEventRecord(c->ev1, c->stream));
  VPS_HIP(c, hipEventSynchronize(c->ev1));
  float ms = 0.f;
  VPS_HIP(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  VPS_HIP(c, timer_flush(c));
  inf.rel_residual_true = bn > 0.0 ? true_rn / bn : 0.0;
  inf.seconds = ms * 1e-3;
  if (info) *info = inf;
  if (result == VPS_E_NOT_CONVERGED) c->err = "maximum number of iterations reached";
  return result;
}

vps_status vps_vcycle_iterate(vps_context* c, const double* b, double* u, int iters, double* res_hist) {
  if (!c || !b || !u) return fail(c, VPS_E_ARG, "null argument");
  if (iters < 0) return fail(c, VPS_E_ARG, "negative iteration count");
  if (vps_status s = need_coef(c)) return s;
  if (vps_status s = need_coarse(c)) return s;
  if (vps_status s = ensure_cg(c)) return s;
  const int L = (int)c->lv.size() - 1;
  const size_t n = c->lv[L].nodes;
  double s2[2];
  for (int it = 0; it <= iters; ++it) {
    VPS_HIP(c, do_operator(c, L, u, b, c->cg_r, VPS_F64));
    if (res_hist) {
      if (vps_status st = dots(c, c->cg_r, c->cg_r, nullptr, nullptr, n, s2)) return st;
      res_hist[it] = std::sqrt(s2[0]);
    }
    if (it == iters) break;
    VPS_HIP(c, do_vcycle(c, c->cg_r, c->cg_z));
    VPS_HIP(c, vps::launch_axpy<double>(1.0, c->cg_z, u, n, c->stream));
  }
  VPS_HIP(c, hipStreamSynchronize(c->stream));
  return VPS_OK;
}

vps_status vps_timing_enable(vps_context* c, int enable) {
  if (!c) return VPS_E_ARG;
  VPS_HIP(c, timer_flush(c));
  c->timer.on = enable != 0;
  if (c->timer.on) {
    c->timer.tot = vps_timing{};
    c->timer.tot.n_levels = (int)c->lv.size();
  }
  return VPS_OK;
}

vps_status vps_timing_get(vps_context* c, vps_timing* out) {
  if (!c || !out) return VPS_E_ARG;
  VPS_HIP(c, timer_flush(c));
  *out = c->timer.tot;
  out->n_levels = (int)c->lv.size();
  return VPS_OK;
}

vps_status vps_sync(vps_context* c) {
  if (!c) return VPS_E_ARG;
  VPS_HIP(c, hipStreamSynchronize(c->stream));
  VPS_HIP(c, hipGetLastError());
  return VPS_OK;
}

}  // extern "C"

// ---- learned part: thin wrappers over the MLP launchers ----
namespace {
vps_status need_mlp_shape(vps_context* c) {
  if (!c) return VPS_E_ARG;
  const int nout = ipow(2 * c->cfg.degree - 1, c->cfg.dim);
  if (nout > vps::kMlpMaxOut)
    return fail(c, VPS_E_UNSUPPORTED, "the MLP supports at most 27 eigenmodes per patch (degree <= 2 in 3D)");
  return VPS_OK;
}
}  // namespace

extern "C" {

vps_status vps_patch_features(vps_context* c, int level, float* x) {
  if (!c || !x) return fail(c, VPS_E_ARG, "null argument");
  if (!level_ok(c, level)) return fail(c, VPS_E_ARG, "invalid level");
  if (c->cfg.coef == VPS_COEF_CONST || !c->coef_set) return fail(c, VPS_E_STATE, "no cell coefficient set");
  const Level& L = c->lv[level];
  VPS_HIP(c, vps::launch_patch_features(L.rho64, L.ncell, c->cfg.dim, x, c->stream));
  return VPS_OK;
}

vps_status vps_patch_rho8(vps_context* c, int level, double* rho8) {
  if (!c || !rho8) return fail(c, VPS_E_ARG, "null argument");
  if (!level_ok(c, level)) return fail(c, VPS_E_ARG, "invalid level");
  if (c->cfg.coef == VPS_COEF_CONST || !c->coef_set) return fail(c, VPS_E_STATE, "no cell coefficient set");
  const Level& L = c->lv[level];
  VPS_HIP(c, vps::launch_patch_rho8(L.rho64, L.ncell, c->cfg.dim, rho8, c->stream));
  return VPS_OK;
}

vps_status vps_rho8_features(vps_context* c, const double* rho8, long long n, float* x) {
  if (!c || (n > 0 && (!rho8 || !x))) return fail(c, VPS_E_ARG, "null argument");
  if (n < 0) return fail(c, VPS_E_ARG, "negative count");
  if (n == 0) return VPS_OK;
  VPS_HIP(c, vps::launch_rho8_features(rho8, n, c->cfg.dim, x, c->stream));
  return VPS_OK;
}

vps_status vps_patch_targets(vps_context* c, const double* rho8, long long n, double* cstar, float* logt) {
  if (!c || (!rho8 && n > 0) || (!cstar && n > 0)) return fail(c, VPS_E_ARG, "null argument");
  if (n < 0) return fail(c, VPS_E_ARG, "negative count");
  if (c->cfg.degree != 2 || c->cfg.dim != 3) return fail(c, VPS_E_UNSUPPORTED, "targets are implemented for Q2 in 3D");
  if (n == 0) return VPS_OK;
  const Level& L = c->lv.back();
  VPS_HIP(c, vps::launch_patch_targets(rho8, n, L.Mh, L.Kh, L.T1.data(), L.lam.data(), cstar, logt, c->stream));
  return VPS_OK;
}

vps_status vps_mlp_forward(vps_context* c, const float* params, const float* x, long long n, float* y, float* act) {
  if (vps_status s = need_mlp_shape(c)) return s;
  if (!c || !params || !x || !y) return fail(c, VPS_E_ARG, "null argument");
  if (n < 0) return fail(c, VPS_E_ARG, "negative count");
  const int nin = 1 << c->cfg.dim, nout = ipow(2 * c->cfg.degree - 1, c->cfg.dim);
  VPS_HIP(c, vps::launch_mlp_forward(params, x, n, nin, nout, y, act, c->stream));
  return VPS_OK;
}

vps_status vps_mlp_loss_grad(vps_context* c, const float* y, const float* t, long long n, float* dy, float* loss) {
  if (vps_status s = need_mlp_shape(c)) return s;
  if (!c || !y || !t || !dy) return fail(c, VPS_E_ARG, "null argument");
  if (n <= 0) return fail(c, VPS_E_ARG, "count must be positive");
  const int nout = ipow(2 * c->cfg.degree - 1, c->cfg.dim);
  if (vps::mlp_ensure(&c->mlp) != hipSuccess) return fail(c, VPS_E_NOMEM, "MLP work allocation failed");
  VPS_HIP(c, vps::launch_mlp_loss_grad(y, t, n, nout, dy, loss, &c->mlp, c->stream));
  return VPS_OK;
}

vps_status vps_mlp_backward(vps_context* c, const float* params, const float* x, const float* act, const float* dy,
                            long long n, float* dparams) {
  if (vps_status s = need_mlp_shape(c)) return s;
  if (!c || !params || !x || !act || !dy || !dparams) return fail(c, VPS_E_ARG, "null argument");
  if (n <= 0) return fail(c, VPS_E_ARG, "count must be positive");
  const int nin = 1 << c->cfg.dim, nout = ipow(2 * c->cfg.degree - 1, c->cfg.dim);
  if (vps::mlp_ensure(&c->mlp) != hipSuccess) return fail(c, VPS_E_NOMEM, "MLP work allocation failed");
  VPS_HIP(c, vps::launch_mlp_backward(params, x, act, dy, n, nin, nout, dparams, &c->mlp, c->stream));
  return VPS_OK;
}

vps_status vps_mlp_backward_noalloc(vps_context* c, const float* params, const float* x, const float* act,
                                    const float* dy, long long n, float* dparams) {
  if (vps_status s = need_mlp_shape(c)) return s;
  if (!c || !params || !x || !act || !dy || !dparams) return fail(c, VPS_E_ARG, "null argument");
  if (n <= 0) return fail(c, VPS_E_ARG, "count must be positive");
  const int nin = 1 << c->cfg.dim, nout = ipow(2 * c->cfg.degree - 1, c->cfg.dim);
  const long long nmax = vps::mlp_noalloc_max_samples(nin, nout);
  if (n > nmax)
    return fail(c, VPS_E_ARG, "vps_mlp_backward_noalloc: " + std::to_string(n) + " samples exceed the " +
                                  std::to_string(nmax) + " its 4 MiB static work memory holds");
  VPS_HIP(c, vps::launch_mlp_backward_noalloc(params, x, act, dy, n, nin, nout, dparams, c->stream));
  return VPS_OK;
}

vps_status vps_mlp_adam(vps_context* c, float* params, const float* g, float* m, float* v, int step, float lr,
                        float b1, float b2, float eps) {
  if (vps_status s = need_mlp_shape(c)) return s;
  if (!c || !params || !g || !m || !v) return fail(c, VPS_E_ARG, "null argument");
  if (step < 1) return fail(c, VPS_E_ARG, "step counts from 1");
  const int nin = 1 << c->cfg.dim, nout = ipow(2 * c->cfg.degree - 1, c->cfg.dim);
  VPS_HIP(c, vps::launch_mlp_adam(params, g, m, v, vps::mlp_param_count(nin, nout), step, lr, b1, b2, eps, c->stream));
  return VPS_OK;
}

vps_status vps_mlp_infer_patches(vps_context* c, int level, const float* params, long long* fallback) {
  if (vps_status s = need_mlp_shape(c)) return s;
  if (!c || !params) return fail(c, VPS_E_ARG, "null argument");
  if (!level_ok(c, level)) return fail(c, VPS_E_ARG, "invalid level");
  if (c->cfg.coef != VPS_COEF_CELL_LEARNED || !c->coef_set)
    return fail(c, VPS_E_STATE, "needs coef = VPS_COEF_CELL_LEARNED and a coefficient");
  Level& L = c->lv[level];
  long long fb = 0;
  if (L.npatch > 0) {
    if (vps::mlp_ensure(&c->mlp) != hipSuccess) return fail(c, VPS_E_NOMEM, "MLP work allocation failed");
    const int nin = 1 << c->cfg.dim, nout = ipow(2 * c->cfg.degree - 1, c->cfg.dim);
    hipError_t e = vps::mlp_infer_patches(L.rho64, L.ncell, c->cfg.dim, params, nin, nout, L.npatch, L.scal, &fb,
                                          &c->mlp, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "mlp_infer_patches");
  }
  c->fallback[level] = fb;
  if (fallback) *fallback = fb;
  return VPS_OK;
}

}  // extern "C"
