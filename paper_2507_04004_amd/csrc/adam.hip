// Sparse Adam over the Gaussian attributes (Sec. "Additional Strategies", a): one Adam step on
// the Gaussians that some view of the pass reached (tile count > 0), none on the others.
//
// One thread per Gaussian walks every plane of every group, so the visibility test (the tile
// counts of all views) is read once per Gaussian. A wavefront that holds no reached Gaussian
// returns before any parameter traffic. Otherwise every lane loads and stores its parameter
// and both moments, reached or not (the others store what they loaded): full-width stores
// leave the L2 as whole lines, where the stores of the reached lanes alone would leave
// partial lines behind. Gradients are loaded for the reached lanes only. HBM-bound: per
// reached Gaussian and plane 16 B are read (param, moments, gradient) and 12 B written.
#include "gs_internal.hpp"

namespace gs {

__device__ __forceinline__ float act_value(float p, int act) {
  if (act == GS_ACT_EXP) return expf(p);
  if (act == GS_ACT_SIGMOID) return 1.0f / (1.0f + expf(-p));
  return p;
}

// d act / d p at p, from the activated value
__device__ __forceinline__ float act_slope(float a, int act) {
  if (act == GS_ACT_EXP) return a;
  if (act == GS_ACT_SIGMOID) return a * (1.0f - a);
  return 1.0f;
}

__global__ __launch_bounds__(256) void k_adam_sparse(AdamArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool in = i < a.n;
  bool reached = in && !a.visible;
  if (in && a.visible)
    for (int v = 0; v < a.n_views; ++v) reached = reached || a.visible[(int64_t)v * a.n + i] > 0u;
  if (!__any(reached)) return;  // uniform per wavefront
  if (!in) return;
  const Planes P(a.n, (uint32_t)i);
  for (int gi = 0; gi < a.n_groups; ++gi) {
    const AdamGroupDev &G = a.group[gi];
#pragma unroll 4
    for (int j = 0; j < G.k; ++j) {
      float p = P.ld(G.param, j), m = P.ld(G.exp_avg, j), v = P.ld(G.exp_avg_sq, j);
      if (reached) {
        const float g = P.ld(G.grad, j) * act_slope(act_value(p, G.act), G.act);
        m = a.beta1 * m + (1.0f - a.beta1) * g;
        v = a.beta2 * v + (1.0f - a.beta2) * (g * g);
        p = p - G.step_size * m / (sqrtf(v) / a.sqrt_bias2 + a.eps);
        if (G.act_out) P.st(G.act_out, j, act_value(p, G.act));
      }
      P.st(G.param, j, p);
      P.st(G.exp_avg, j, m);
      P.st(G.exp_avg_sq, j, v);
    }
  }
}

hipError_t launch_adam_sparse(const AdamArgs &a, hipStream_t st) {
  if (a.n <= 0 || a.n_groups == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adam_sparse, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace gs
