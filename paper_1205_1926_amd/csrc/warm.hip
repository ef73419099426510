// Learned warm start of the dual PCGP: per-interface-node features, targets
// and the candidate multiplier built from the network's prediction.
//
// An interface node carries up to 21 multiplier rows (7 per component: the
// Helmert gluing rows of a node shared by up to 8 subdomains, or one
// Dirichlet row per copy).  Features of node q (31 values):
//   [0, 3)   direction of the load increment (unit vector);
//   [3, 24)  previous converged multipliers of the node's rows / s_lam;
//   24       mean hardening kappa over the Gauss points of the elements
//            around the node (all subdomain copies), times H / sigma_y;
//   [25, 31) one-hot node class (gluing with 2/4/8 copies, Dirichlet
//            with 1/2/4 copies).
// Targets: (lambda_next - lambda_prev) / s_lam on the node's rows, with
// s_lam = |load increment| * element face area (a nodal force scale).
#include "kernels.h"

namespace tfeti {

__global__ void warm_features_kernel(int64_t n, const int32_t* __restrict__ rows, const int8_t* __restrict__ cls,
                                     const int32_t* __restrict__ erp, const int32_t* __restrict__ elems,
                                     const double* __restrict__ kappa, const double* __restrict__ lam_prev,
                                     double d0, double d1, double d2, double inv_slam, double kscale,
                                     float* __restrict__ X, float* __restrict__ Mk) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  float* x = X + 31 * q;
  x[0] = (float)d0;
  x[1] = (float)d1;
  x[2] = (float)d2;
  for (int s = 0; s < 21; ++s) {
    const int32_t r = rows[21 * q + s];
    x[3 + s] = r >= 0 ? (float)(lam_prev ? lam_prev[r] * inv_slam : 0.0) : 0.f;
    if (Mk) Mk[21 * q + s] = r >= 0 ? 1.f : 0.f;
  }
  double ks = 0.0;
  const int32_t e0 = erp[q], e1 = erp[q + 1];
  for (int32_t e = e0; e < e1; ++e)
    for (int g = 0; g < 8; ++g) ks += kappa[8 * (int64_t)elems[e] + g];
  x[24] = e1 > e0 ? (float)(ks / (8.0 * (e1 - e0)) * kscale) : 0.f;
  for (int c = 0; c < 6; ++c) x[25 + c] = (cls[q] == c) ? 1.f : 0.f;
}

__global__ void warm_targets_kernel(int64_t n, const int32_t* __restrict__ rows, const double* __restrict__ lam_prev,
                                    const double* __restrict__ lam_next, double inv_slam, float* __restrict__ T) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  for (int s = 0; s < 21; ++s) {
    const int32_t r = rows[21 * q + s];
    T[21 * q + s] = r >= 0 ? (float)((lam_next[r] - (lam_prev ? lam_prev[r] : 0.0)) * inv_slam) : 0.f;
  }
}

// every multiplier row belongs to exactly one (node, slot), so this writes
// the whole candidate
__global__ void warm_apply_kernel(int64_t n, const int32_t* __restrict__ rows, const double* __restrict__ lam_prev,
                                  const float* __restrict__ Y, double slam, double* __restrict__ out) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  for (int s = 0; s < 21; ++s) {
    const int32_t r = rows[21 * q + s];
    if (r >= 0) out[r] = (lam_prev ? lam_prev[r] : 0.0) + (double)Y[21 * q + s] * slam;
  }
}

void launch_warm_features(const WarmMaps& W, const double* kappa, const double* lam_prev, const double dir[3],
                          double inv_slam, double kscale, float* X, float* Mk, hipStream_t st) {
  if (W.n <= 0) return;
  warm_features_kernel<<<dim3((unsigned)((W.n + 127) / 128)), dim3(128), 0, st>>>(
      W.n, W.rows, W.cls, W.erp, W.elems, kappa, lam_prev, dir[0], dir[1], dir[2], inv_slam, kscale, X, Mk);
}

void launch_warm_targets(const WarmMaps& W, const double* lam_prev, const double* lam_next, double inv_slam, float* T,
                         hipStream_t st) {
  if (W.n <= 0) return;
  warm_targets_kernel<<<dim3((unsigned)((W.n + 127) / 128)), dim3(128), 0, st>>>(W.n, W.rows, lam_prev, lam_next,
                                                                                 inv_slam, T);
}

void launch_warm_apply(const WarmMaps& W, const double* lam_prev, const float* Y, double slam, double* out,
                       hipStream_t st) {
  if (W.n <= 0) return;
  warm_apply_kernel<<<dim3((unsigned)((W.n + 127) / 128)), dim3(128), 0, st>>>(W.n, W.rows, lam_prev, Y, slam, out);
}

}  // namespace tfeti
