// Photometric tracking (camera factor option 2, eq:tracking_loss): the device side of the
// pose loop. With the map frozen, every iteration renders at the current pose, takes
// L = w_1 mean |C_hat - C| + w_s D-SSIM, differentiates it to the 6-DoF pose tangent
// xi = (rho, phi) of the left perturbation T_cw <- Exp(xi) T_cw, and turns that gradient into
// an Adam step delta applied as T_cw <- Exp(delta) T_cw (the parameter is reset to zero after
// each update; the moments and bias correction run over the iterations).
//
// The pose lives in device memory for the whole loop: a float64 master copy, and the float32
// rotation, translation and camera centre that the projection kernels read, so the loop
// needs no host round trip and can be captured into one graph.
#include <cmath>

#include "gs_internal.hpp"

namespace gs {

namespace {

__device__ void hat3(const double w[3], double P[9]) {
  P[0] = 0.0;   P[1] = -w[2]; P[2] = w[1];
  P[3] = w[2];  P[4] = 0.0;   P[5] = -w[0];
  P[6] = -w[1]; P[7] = w[0];  P[8] = 0.0;
}

__device__ void mul3(const double A[9], const double B[9], double C[9]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

// float32 copies for the kernels: R, t, and the camera centre -R^T t
__device__ void publish_pose(const double R[9], const double t[3], float *pose) {
  for (int i = 0; i < 9; ++i) pose[i] = (float)R[i];
  for (int i = 0; i < 3; ++i) pose[9 + i] = (float)t[i];
  for (int i = 0; i < 3; ++i) pose[12 + i] = (float)(-(R[i] * t[0] + R[3 + i] * t[1] + R[6 + i] * t[2]));
  pose[15] = 0.f;
}

__device__ void publish(const TrackState &s, float *pose) { publish_pose(s.R, s.t, pose); }

// Left update (R, t) <- Exp(d) (R0, t0), d = (rho, phi): closed-form SE(3) exponential
// R = I + A P + B P^2, V = I + B P + C P^2 with P = phi^ (series for small angles).
__device__ void left_exp(const double d[6], const double R0[9], const double t0[3], double R[9], double t[3]) {
  const double th2 = d[3] * d[3] + d[4] * d[4] + d[5] * d[5];
  const double th = sqrt(th2);
  double A, B, C;
  if (th < 1e-5) {
    A = 1.0 - th2 / 6.0;
    B = 0.5 - th2 / 24.0;
    C = 1.0 / 6.0 - th2 / 120.0;
  } else {
    const double sn = sin(th), cs = cos(th);
    A = sn / th;
    B = (1.0 - cs) / th2;
    C = (th - sn) / (th2 * th);
  }
  double P[9], P2[9];
  hat3(d + 3, P);
  mul3(P, P, P2);
  double dR[9], V[9];
  for (int i = 0; i < 9; ++i) {
    const double I = (i % 4 == 0) ? 1.0 : 0.0;
    dR[i] = I + A * P[i] + B * P2[i];
    V[i] = I + B * P[i] + C * P2[i];
  }
  mul3(dR, R0, R);
  for (int i = 0; i < 3; ++i)
    t[i] = dR[3 * i] * t0[0] + dR[3 * i + 1] * t0[1] + dR[3 * i + 2] * t0[2] +
           (V[3 * i] * d[0] + V[3 * i + 1] * d[1] + V[3 * i + 2] * d[2]);
}

}  // namespace

// One lane sets up the loop state: master pose from the caller's camera, zero moments.
__global__ void k_track_init(TrackState *__restrict__ s, TrackPose p0) {
  if (threadIdx.x != 0) return;
  TrackState st;
  for (int i = 0; i < 9; ++i) st.R[i] = p0.R[i];
  for (int i = 0; i < 3; ++i) st.t[i] = p0.t[i];
  for (int i = 0; i < 6; ++i) st.m[i] = st.v[i] = 0.0;
  st.max_pairs = 0;
  publish(st, st.pose);
  for (int i = 0; i < 6; ++i) st.grad[i] = 0.f;
  st.loss[0] = st.loss[1] = 0.f;
  *s = st;
}

// Iteration k (1-based): record the trace, take the Adam step on the gradient the backward
// left in s->grad, apply Exp(delta) on the left, publish the new pose. One lane, float64.
__global__ void k_track_step(TrackState *__restrict__ s, TrackStepArgs a, const int64_t *__restrict__ num_pairs,
                             float *__restrict__ trace, float *__restrict__ pose_out) {
  if (threadIdx.x != 0) return;
  TrackState st = *s;
  if (trace) {
    float *r = trace + (int64_t)(a.k - 1) * kTrackTraceStride;
    for (int i = 0; i < 12; ++i) r[i] = st.pose[i];
    for (int i = 0; i < 6; ++i) r[12 + i] = st.grad[i];
    r[18] = st.loss[0];
    r[19] = st.loss[1];
  }
  st.max_pairs = max(st.max_pairs, *num_pairs);
  double d[6];
  for (int i = 0; i < 6; ++i) {
    const double g = (double)st.grad[i];
    st.m[i] = a.beta1 * st.m[i] + (1.0 - a.beta1) * g;
    st.v[i] = a.beta2 * st.v[i] + (1.0 - a.beta2) * (g * g);
    const double mh = st.m[i] / a.bias1, vh = st.v[i] / a.bias2;
    d[i] = -a.lr[i] * mh / (sqrt(vh) + a.eps);
  }
  double R[9], t[3];
  left_exp(d, st.R, st.t, R, t);
  for (int i = 0; i < 9; ++i) st.R[i] = R[i];
  for (int i = 0; i < 3; ++i) st.t[i] = t[i];
  publish(st, st.pose);
  *s = st;
  if (pose_out)
    for (int i = 0; i < 12; ++i) pose_out[i] = st.pose[i];
}

// One lane: the pose Exp(xi) (R0, t0) of a tangent xi (float32 [6], device) as the float32
// R (9), t (3) and camera centre (3) the projection kernels read through a device pointer.
__global__ void k_pose_left_update(TrackPose p0, const float *__restrict__ xi, float *__restrict__ pose) {
  if (threadIdx.x != 0) return;
  double d[6];
  for (int i = 0; i < 6; ++i) d[i] = (double)xi[i];
  double R[9], t[3];
  left_exp(d, p0.R, p0.t, R, t);
  publish_pose(R, t, pose);
}

hipError_t launch_pose_left_update(const TrackPose &p0, const float *xi, float *pose, hipStream_t st) {
  hipLaunchKernelGGL(k_pose_left_update, dim3(1), dim3(64), 0, st, p0, xi, pose);
  return hipGetLastError();
}

hipError_t launch_track_init(TrackState *s, const TrackPose &p0, hipStream_t st) {
  hipLaunchKernelGGL(k_track_init, dim3(1), dim3(64), 0, st, s, p0);
  return hipGetLastError();
}

hipError_t launch_track_step(TrackState *s, const TrackStepArgs &a, const int64_t *num_pairs, float *trace,
                             float *pose_out, hipStream_t st) {
  hipLaunchKernelGGL(k_track_step, dim3(1), dim3(64), 0, st, s, a, num_pairs, trace, pose_out);
  return hipGetLastError();
}

}  // namespace gs
