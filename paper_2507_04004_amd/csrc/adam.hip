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

constexpr int kAdamBatch = 8;  // planes whose loads are in flight together

__global__ __launch_bounds__(256) void k_adam_sparse(AdamArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool in = i < a.n;
  bool reached = in && !a.visible;
  if (in && a.visible)
    for (int v = 0; v < a.n_views; ++v) reached = reached || a.visible[(int64_t)v * a.n + i] > 0u;
  if (!__any(reached)) return;  // uniform per wavefront
  if (!in) return;
  const Planes P(a.n, (uint32_t)i);
  // Planes are taken kAdamBatch at a time, every load of a batch issued before its first
  // store: the buffer stores may alias any plane, so a load placed after a store waits for it,
  // and one plane per round trip would leave a wavefront with four loads in flight.
  for (int gi = 0; gi < a.n_groups; ++gi) {
    const AdamGroupDev &G = a.group[gi];
    for (int j0 = 0; j0 < G.k; j0 += kAdamBatch) {
      const int nb = min(kAdamBatch, G.k - j0);  // uniform
      float p[kAdamBatch], m[kAdamBatch], v[kAdamBatch], g[kAdamBatch];
#pragma unroll
      for (int u = 0; u < kAdamBatch; ++u) {
        if (u < nb) {
          p[u] = P.ld(G.param, j0 + u);
          m[u] = P.ld(G.exp_avg, j0 + u);
          v[u] = P.ld(G.exp_avg_sq, j0 + u);
          g[u] = reached ? P.ld(G.grad, j0 + u) : 0.f;
        }
      }
#pragma unroll
      for (int u = 0; u < kAdamBatch; ++u) {
        if (u >= nb) break;
        if (reached) {
          const float gr = g[u] * act_slope(act_value(p[u], G.act), G.act);
          m[u] = a.beta1 * m[u] + (1.0f - a.beta1) * gr;
          v[u] = a.beta2 * v[u] + (1.0f - a.beta2) * (gr * gr);
          p[u] = p[u] - G.step_size * m[u] / (sqrtf(v[u]) / a.sqrt_bias2 + a.eps);
          if (G.act_out) P.st(G.act_out, j0 + u, act_value(p[u], G.act));
        }
        P.st(G.param, j0 + u, p[u]);
        P.st(G.exp_avg, j0 + u, m[u]);
        P.st(G.exp_avg_sq, j0 + u, v[u]);
      }
    }
  }
}

hipError_t launch_adam_sparse(const AdamArgs &a, hipStream_t st) {
  if (a.n <= 0 || a.n_groups == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adam_sparse, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace gs
