// Launchers of the learned-scaling kernels (library-internal).
//
// MLP n_in -> 64 (tanh) -> 64 (tanh) -> n_out, FP32; flat parameters
// W1 (64 x n_in, row-major), b1, W2 (64 x 64), b2, W3 (n_out x 64), b3.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

namespace vps {

constexpr int kMlpHidden = 64;
constexpr int kMlpMaxIn = 8;
constexpr int kMlpMaxOut = 27;

__host__ __device__ inline int mlp_param_count(int nin, int nout) {
  return kMlpHidden * nin + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden + nout * kMlpHidden + nout;
}

struct MlpWork {
  float* delta = nullptr;     // per-sample back-propagated signals
  size_t delta_cap = 0;       // floats
  float* partial = nullptr;   // split partial gradients / loss partial sums
  size_t partial_cap = 0;     // floats
  int* counter = nullptr;     // fallback counter
  int* hcounter = nullptr;    // pinned host copy
};

hipError_t mlp_ensure(MlpWork* w);
void mlp_free(MlpWork* w);

hipError_t launch_patch_features(const double* rho, int ncell, int dim, float* x, hipStream_t s);
hipError_t launch_patch_rho8(const double* rho, int ncell, int dim, double* rho8, hipStream_t s);
hipError_t launch_rho8_features(const double* rho8, long long n, int dim, float* x, hipStream_t s);

// Exact targets for Q2 patches in 3D (see vps_patch_targets).
hipError_t launch_patch_targets(const double* rho8, long long n, const std::vector<double>* Mh,
                                const std::vector<double>* Kh, const double* T1, const double* lam, double* cstar,
                                float* log_target, hipStream_t s);

// Exact dense local solvers of Q2 patches (3D): binv[j] = A_j(rho)^{-1} for every patch of a level
// (npatch x 27 x 27 FP64), from the level's half-cell 1D matrices; and one color step u_I += B_j r_I.
hipError_t launch_exact_inverses(const double* rho, int ncell, const std::vector<double>* Mh,
                                 const std::vector<double>* Kh, double* binv, hipStream_t s);
hipError_t launch_exact_apply(double* u, const double* r, const double* binv, int n1, int ncell, int color,
                              hipStream_t s);

hipError_t launch_mlp_forward(const float* params, const float* x, long long n, int nin, int nout, float* y,
                              float* act, hipStream_t s);
hipError_t launch_mlp_loss_grad(const float* y, const float* t, long long n, int nout, float* dy, float* loss,
                                MlpWork* w, hipStream_t s);
hipError_t launch_mlp_backward(const float* params, const float* x, const float* act, const float* dy, long long n,
                               int nin, int nout, float* dparams, MlpWork* w, hipStream_t s);
// Allocation-free form of launch_mlp_backward: the work memory is a static device array of 4 MiB
// (one per GPU, shared by every call on it); n <= mlp_noalloc_max_samples(nin, nout).
// mlp_scratch_setup() must have run once on the current device (vps_create does it).
hipError_t mlp_scratch_setup();
long long mlp_noalloc_max_samples(int nin, int nout);
hipError_t launch_mlp_backward_noalloc(const float* params, const float* x, const float* act, const float* dy,
                                       long long n, int nin, int nout, float* dparams, hipStream_t s);
hipError_t launch_mlp_adam(float* params, const float* g, float* m, float* v, int np, int step, float lr, float b1,
                           float b2, float eps, hipStream_t s);
// features -> MLP -> clamp(exp(y), 1/4, 4) per patch of a level, fallback 1 on non-finite output.
hipError_t mlp_infer_patches(const double* rho, int ncell, int dim, const float* params, int nin, int nout,
                             long long npatch, float* scal, long long* fallback, MlpWork* w, hipStream_t s);

}  // namespace vps
