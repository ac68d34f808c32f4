// Fluid half of the staggered (sequential) iteration: the decoupled fluid
// equation D dP = -R_p with the opening held (D = dR_p/dP, the Poiseuille
// flux operator alone), closed by one essential pressure condition per
// instance, solved with the dense inverse of the pressure block.
#include "hf_internal.h"

namespace hf {

// row `node[b]` of instance b's copy W of D becomes the identity row and its
// residual entry P[node] - value; one workgroup per instance
__global__ void k_stag_dirichlet(const int32_t *__restrict__ poff, const int64_t *__restrict__ doff,
                                 const int32_t *__restrict__ node, const double *__restrict__ value,
                                 const double *__restrict__ p, double *__restrict__ W,
                                 double *__restrict__ Rp) {
  const int b = blockIdx.x;
  const int32_t p0 = poff[b];
  const int nb = poff[b + 1] - p0;
  if (nb == 0) return;
  const int i = node[b];
  double *row = W + doff[b] + (int64_t)i * nb;
  for (int j = threadIdx.x; j < nb; j += blockDim.x) row[j] = (j == i) ? 1.0 : 0.0;
  if (threadIdx.x == 0) Rp[p0 + i] = p[p0 + i] - value[b];
}

// dP_i = -sum_j Winv_b[i][j] R_p[p0 + j], one wave per pressure row
__global__ __launch_bounds__(64) void k_stag_dp(const int32_t *__restrict__ pinst,
                                                const int32_t *__restrict__ poff,
                                                const int64_t *__restrict__ doff,
                                                const double *__restrict__ Winv,
                                                const double *__restrict__ Rp, double *__restrict__ dp) {
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x;
  const int b = pinst[i];
  const int64_t p0 = poff[b], nb = poff[b + 1] - p0;
  const double *row = Winv + doff[b] + (i - p0) * nb;
  double acc = 0.0;
  for (int64_t j = lane; j < nb; j += 64) acc += row[j] * Rp[p0 + j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) dp[i] = -acc;
}

hipError_t launch_stag_dirichlet(const KParams &kp, const int32_t *node, const double *value,
                                 const double *p, double *W, double *Rp, hipStream_t st) {
  if (!kp.s.n_p) return hipSuccess;
  hipLaunchKernelGGL(k_stag_dirichlet, dim3(kp.n_inst), dim3(256), 0, st, kp.poff, kp.doff, node, value, p,
                     W, Rp);
  return hipGetLastError();
}

hipError_t launch_stag_dp(const KParams &kp, const double *Winv, const double *Rp, double *dp,
                          hipStream_t st) {
  if (!kp.s.n_p) return hipSuccess;
  hipLaunchKernelGGL(k_stag_dp, dim3((unsigned)kp.s.n_p), dim3(64), 0, st, kp.pinst, kp.poff, kp.doff, Winv,
                     Rp, dp);
  return hipGetLastError();
}

}  // namespace hf
