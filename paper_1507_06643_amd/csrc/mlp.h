// Surrogate for the inverse internal equation of state theta(eps).
//
// Network: x = (ln eps - in_c)/in_s, h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2),
// y = W3 . h2 + b3, theta = exp(out_c + out_s y); 32 hidden units per layer,
// weights packed W1[32] b1[32] W2[32][32] b2[32] W3[32] b3 (1153 values).
//
// Inference: the 32x32 layer runs on the matrix cores in BF16 with FP32
// accumulation (the input and output layers, on the vector units, use the
// FP32 weights) as H2^T = W2 H1^T with one v_mfma_f32_32x32x16_bf16 per
// (32 particles x 16 inputs) block: the weights are the A operand (constant),
// each lane builds its B-operand column of tanh(W1 x + b1) for the particle it
// serves, and the accumulator leaves every lane with 16 hidden units of one
// particle, so the output layer is a 16-term dot product plus one cross-half
// shuffle.
//
// Training runs in FP32 on the GPU: forward and backward per sample in
// registers, per-block gradient sums in a fixed order through LDS, a second
// kernel adds the block partials in block order and applies Adam.  Samples
// are theta log-uniform in the training range, eps = eps(theta) from the EOS.
#pragma once

#include <cmath>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "common.h"
#include "eos.h"

namespace dpde {

constexpr int kH = 32;
constexpr int kNParam = kH + kH + kH * kH + kH + kH + 1;  // 1153
constexpr int OFF_W1 = 0, OFF_B1 = kH, OFF_W2 = 2 * kH, OFF_B2 = OFF_W2 + kH * kH;
constexpr int OFF_W3 = OFF_B2 + kH, OFF_B3 = OFF_W3 + kH;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

struct MlpState {
  bool trained = false;
  float* w = nullptr;       // FP32 master weights
  uint16_t* wb = nullptr;   // BF16 bit patterns used by inference
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  float* gpart = nullptr;   // per-block gradient partials
  double* lpart = nullptr;  // per-block loss partials
  float* loss = nullptr;    // loss per iteration
  float* gsum = nullptr;    // summed gradient (gradient checks)
  float* xs = nullptr;      // training inputs
  float* ts = nullptr;      // training targets
  int64_t nsamp = 0;
  int64_t loss_cap = 0;
  int gblocks = 0;
  double norm[4] = {0, 1, 0, 1};  // in_c, in_s, out_c, out_s
  double eps_lo = 0, eps_hi = 0;
  std::vector<void*> allocs;
};

// ---- conversions ----------------------------------------------------------------
__host__ __device__ inline uint16_t f32_to_bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) {
  return __uint_as_float((uint32_t)b << 16);
}

__device__ __forceinline__ float fast_tanh(float x) {
  // tanh x = 1 - 2/(e^{2x} + 1); e^{2x} = 2^{2x log2 e}
  const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * x);
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

// ---- inference: every lane of the wave must call; returns this lane's y ---------
// The 32x32 layer is the matrix-core product: W2 and the hidden activations
// enter it in BF16.  The input and output layers (vectors, evaluated on the
// vector units) keep the FP32 master weights.
// 32 particles: lane l serves particle l % 32 (both half-waves pass that
// particle's x) and every lane gets that particle's y.
__device__ __forceinline__ float mlp_wave32(const float* __restrict__ wf,
                                            const uint16_t* __restrict__ wb, float xp) {
  const int l = threadIdx.x % kWave;
  const int half = l >> 5, col = l & 31;
  bf16x8 a[2];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks)
#pragma unroll
    for (int e = 0; e < 8; ++e)
      a[ks][e] = __builtin_bit_cast(__bf16, wb[OFF_W2 + col * kH + ks * 16 + 8 * half + e]);
  f32x16 acc = {};
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
    bf16x8 b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = ks * 16 + 8 * half + e;
      const float h = fast_tanh(wf[OFF_W1 + k] * xp + wf[OFF_B1 + k]);
      b[e] = __builtin_bit_cast(__bf16, f32_to_bf16_bits(h));
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ks], b, acc, 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int u = 8 * (r >> 2) + 4 * half + (r & 3);
    s += wf[OFF_W3 + u] * fast_tanh(acc[r] + wf[OFF_B2 + u]);
  }
  s += __shfl_xor(s, 32, kWave);
  return s + wf[OFF_B3];
}

// 64 particles: lane l passes the x of particle l and gets its y.
__device__ __forceinline__ float mlp_wave(const float* __restrict__ wf,
                                          const uint16_t* __restrict__ wb, float x) {
  const int l = threadIdx.x % kWave;
  const int half = l >> 5, col = l & 31;
  float y[2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) y[mb] = mlp_wave32(wf, wb, __shfl(x, 32 * mb + col, kWave));
  return half ? y[1] : y[0];
}

struct MlpDev {
  const float* wf;     // FP32 master weights (input and output layers)
  const uint16_t* wb;  // BF16 copy (the matrix-core layer W2)
  double in_c, in_s, out_c, out_s, eps_lo, eps_hi;
};

// theta (OUT_INV = 0) or 1/theta (OUT_INV = 1) for n energies.  mode 1: the
// network inside [eps_lo, eps_hi], Newton outside; mode 2: Newton started
// from the network's estimate (or the asymptote outside the range); mode 0:
// Newton alone.  No lane leaves before the matrix-core step.
// Network input for eps: normalised log, clamped to the training interval.
__device__ __forceinline__ float mlp_input(const MlpDev& m, double e) {
  double xd = (log(e > 0.0 ? e : 1.0) - m.in_c) / m.in_s;
  xd = xd < -1.0 ? -1.0 : (xd > 1.0 ? 1.0 : xd);
  return (float)xd;
}

// theta from the network output y (modes 1, 2) or by Newton (mode 0, and
// outside the training range in mode 1).
__device__ __forceinline__ double theta_from_net(const Phys& P, const MlpDev& m, int mode,
                                                 double e, float y, int& it) {
  it = 0;
  if (P.eos == 0) return e / P.cv;
  const bool in_range = e >= m.eps_lo && e <= m.eps_hi;
  const double th_net = mode != 0 ? exp(m.out_c + m.out_s * (double)y) : 0.0;
  if (mode == 1 && in_range) return th_net;
  return theta_newton_dev(P, e, (mode == 2 && in_range) ? th_net : theta_start_dev(P, e), it);
}

template <int OUT_INV>
__global__ __launch_bounds__(256) void k_theta(const double* __restrict__ eps, double* __restrict__ out,
                                               int64_t ostride, int32_t* __restrict__ iters,
                                               int64_t n, Phys P, MlpDev m, int mode,
                                               uint32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  const double e = valid ? eps[i] : 1.0;
  float y = 0.0f;
  if (P.eos != 0 && mode != 0) y = mlp_wave(m.wf, m.wb, mlp_input(m, e));  // uniform
  int it;
  const double th = theta_from_net(P, m, mode, e, y, it);
  if (!valid) return;
  if (!(e > 0.0)) {
    if (status) atomicOr(status, ST_NEG_EINT);
    return;
  }
  if (!(th > 0.0) || !isfinite(th)) {
    if (status) atomicOr(status, ST_EOS);
  }
  out[i * ostride] = OUT_INV ? 1.0 / th : th;
  if (iters) iters[i] = it;
}

__global__ void k_eos_energy(const double* __restrict__ theta, double* __restrict__ eps, int64_t n,
                             Phys P) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) eps[i] = eos_energy_dev(P, theta[i]);
}

// y for normalised inputs (test hook for the inference path).
__global__ __launch_bounds__(256) void k_mlp_eval(const float* __restrict__ wf,
                                                  const uint16_t* __restrict__ wb,
                                                  const float* __restrict__ x, float* __restrict__ y,
                                                  int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const float xi = i < n ? x[i] : 0.0f;
  const float v = mlp_wave(wf, wb, xi);
  if (i < n) y[i] = v;
}

// ---- training ---------------------------------------------------------------------
constexpr int kTrainThreads = 128;
constexpr int kLd = kH + 1;  // padded LDS row

// Training samples: theta log-uniform in [lo, hi] from Philox words keyed by
// the seed (counter = sample index), eps = eps(theta).
__global__ void k_mlp_samples(uint64_t seed, int64_t n, double lnlo, double lnhi, Phys P,
                              double in_c, double in_s, double out_c, double out_s,
                              float* __restrict__ xs, float* __restrict__ ts) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  uint32_t w0 = (uint32_t)k, w1 = (uint32_t)(k >> 32), w2 = 0x534D504Cu, w3 = 0u;
  philox4x32_10(w0, w1, w2, w3, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double u = ((double)w0 + 0.5) * 2.3283064365386963e-10;
  const double lt = lnlo + u * (lnhi - lnlo);
  const double th = exp(lt);
  const double e = eos_energy_dev(P, th);
  xs[k] = (float)((log(e) - in_c) / in_s);
  ts[k] = (float)((lt - out_c) / out_s);
}

// Forward + backward of nb samples starting at sample `begin` (mod nsamp), in
// chunks of kTrainThreads per block; block partial gradients of the mean
// squared error scaled by inv_batch.
__global__ __launch_bounds__(kTrainThreads) void k_mlp_fwd_bwd(
    const float* __restrict__ w, const float* __restrict__ xs, const float* __restrict__ ts,
    int64_t nsamp, int64_t begin, int64_t nb, float inv_batch, float* __restrict__ gpart,
    double* __restrict__ lpart) {
  __shared__ float H1[kTrainThreads * kLd];
  __shared__ float H2[kTrainThreads * kLd];
  __shared__ float D1[kTrainThreads * kLd];
  __shared__ float D2[kTrainThreads * kLd];
  __shared__ float X[kTrainThreads];
  __shared__ float DY[kTrainThreads];
  __shared__ double red[kTrainThreads / kWave];
  const int tid = threadIdx.x;
  const float* W1 = w + OFF_W1;
  const float* B1 = w + OFF_B1;
  const float* W2 = w + OFF_W2;
  const float* B2 = w + OFF_B2;
  const float* W3 = w + OFF_W3;
  const float b3 = w[OFF_B3];
  constexpr int kPer = (kNParam + kTrainThreads - 1) / kTrainThreads;
  float acc[kPer];
#pragma unroll
  for (int c = 0; c < kPer; ++c) acc[c] = 0.0f;
  double lsum = 0.0;
  // this block's share of the nb samples
  const int64_t per_block = (nb + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per_block;
  const int64_t b1 = b0 + per_block < nb ? b0 + per_block : nb;
  for (int64_t c0 = b0; c0 < b1; c0 += kTrainThreads) {
    const int64_t s = c0 + tid;
    const bool live = s < b1;
    float x = 0.0f, t = 0.0f;
    if (live) {
      const int64_t k = (begin + s) % nsamp;
      x = xs[k];
      t = ts[k];
    }
    float h1[kH], h2[kH];
#pragma unroll
    for (int a = 0; a < kH; ++a) h1[a] = tanhf(W1[a] * x + B1[a]);
    float y = b3;
#pragma unroll 4
    for (int a = 0; a < kH; ++a) {
      float z = B2[a];
#pragma unroll
      for (int b = 0; b < kH; ++b) z += W2[a * kH + b] * h1[b];
      h2[a] = tanhf(z);
      y += W3[a] * h2[a];
    }
    const float err = live ? (y - t) : 0.0f;
    lsum += (double)err * (double)err;
    const float dy = 2.0f * err * inv_batch;
    float d2[kH];
#pragma unroll
    for (int a = 0; a < kH; ++a) d2[a] = dy * W3[a] * (1.0f - h2[a] * h2[a]);
#pragma unroll 4
    for (int b = 0; b < kH; ++b) {
      float z = 0.0f;
#pragma unroll
      for (int a = 0; a < kH; ++a) z += W2[a * kH + b] * d2[a];
      D1[tid * kLd + b] = z * (1.0f - h1[b] * h1[b]);
    }
#pragma unroll
    for (int a = 0; a < kH; ++a) {
      H1[tid * kLd + a] = live ? h1[a] : 0.0f;
      H2[tid * kLd + a] = live ? h2[a] : 0.0f;
      D2[tid * kLd + a] = d2[a];
    }
    X[tid] = x;
    DY[tid] = dy;
    __syncthreads();
    const int rows = (int)((b1 - c0) < kTrainThreads ? (b1 - c0) : kTrainThreads);
#pragma unroll
    for (int c = 0; c < kPer; ++c) {
      const int p = tid + c * kTrainThreads;
      if (p >= kNParam) break;
      float g = 0.0f;
      if (p < OFF_B1) {
        for (int r = 0; r < rows; ++r) g += D1[r * kLd + p] * X[r];
      } else if (p < OFF_W2) {
        for (int r = 0; r < rows; ++r) g += D1[r * kLd + (p - OFF_B1)];
      } else if (p < OFF_B2) {
        const int a = (p - OFF_W2) / kH, b = (p - OFF_W2) % kH;
        for (int r = 0; r < rows; ++r) g += D2[r * kLd + a] * H1[r * kLd + b];
      } else if (p < OFF_W3) {
        for (int r = 0; r < rows; ++r) g += D2[r * kLd + (p - OFF_B2)];
      } else if (p < OFF_B3) {
        for (int r = 0; r < rows; ++r) g += DY[r] * H2[r * kLd + (p - OFF_W3)];
      } else {
        for (int r = 0; r < rows; ++r) g += DY[r];
      }
      acc[c] += g;
    }
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int p = tid + c * kTrainThreads;
    if (p < kNParam) gpart[(int64_t)blockIdx.x * kNParam + p] = acc[c];
  }
  double v[1] = {lsum};
  block_sum<1>(v, red);
  if (tid == 0) lpart[blockIdx.x] = v[0];
}

// Sum the block partials in block order; optionally apply one Adam step
// (beta1 0.9, beta2 0.999, eps 1e-8) and refresh the BF16 copy.
__global__ void k_mlp_reduce_adam(const float* __restrict__ gpart, const double* __restrict__ lpart,
                                  int nblocks, int64_t batch, float* __restrict__ w,
                                  float* __restrict__ m, float* __restrict__ v,
                                  uint16_t* __restrict__ wb, float lr, float bc1, float bc2,
                                  int update, float* __restrict__ gsum, float* __restrict__ loss_out) {
  for (int p = threadIdx.x; p < kNParam; p += blockDim.x) {
    float g = 0.0f;
    for (int b = 0; b < nblocks; ++b) g += gpart[(int64_t)b * kNParam + p];
    if (gsum) gsum[p] = g;
    if (update) {
      const float mm = 0.9f * m[p] + 0.1f * g;
      const float vv = 0.999f * v[p] + 0.001f * g * g;
      m[p] = mm;
      v[p] = vv;
      const float wn = w[p] - lr * (mm / bc1) / (sqrtf(vv / bc2) + 1e-8f);
      w[p] = wn;
      wb[p] = f32_to_bf16_bits(wn);
    }
  }
  if (threadIdx.x == 0 && loss_out) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += lpart[b];
    *loss_out = (float)(s / (double)batch);
  }
}

__global__ void k_to_bf16(const float* __restrict__ w, uint16_t* __restrict__ wb, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wb[i] = f32_to_bf16_bits(w[i]);
}

// ---- host helpers -------------------------------------------------------------------
inline double eos_energy_host(const Phys& P, double th) {
  if (P.eos == 0) return P.cv * th;
  const double x = P.eos_omega / th;
  return P.eos_n * P.eos_omega * std::exp(-x) / (-std::expm1(-x)) + P.eos_c0 * th;
}

template <typename T>
inline int mlp_alloc(MlpState& s, T** p, size_t count) {
  void* ptr = nullptr;
  if (hipMalloc(&ptr, (count ? count : 1) * sizeof(T)) != hipSuccess) return DPDE_ENOMEM;
  s.allocs.push_back(ptr);
  *p = (T*)ptr;
  return DPDE_OK;
}

inline void mlp_release(MlpState& s) {
  for (void* p : s.allocs) (void)hipFree(p);
  s.allocs.clear();
  s = MlpState{};
}

inline int mlp_ensure_weights(MlpState& s) {
  if (s.w) return DPDE_OK;
  int rc;
  if ((rc = mlp_alloc(s, &s.w, kNParam)) || (rc = mlp_alloc(s, &s.wb, kNParam)) ||
      (rc = mlp_alloc(s, &s.adam_m, kNParam)) || (rc = mlp_alloc(s, &s.adam_v, kNParam)) ||
      (rc = mlp_alloc(s, &s.gsum, kNParam)))
    return rc;
  return DPDE_OK;
}

inline MlpDev mlp_dev(const MlpState& s) {
  return MlpDev{s.w, s.wb, s.norm[0], s.norm[1], s.norm[2], s.norm[3], s.eps_lo, s.eps_hi};
}

// Copy the normalisation into the physics block used by the step kernels.
inline void mlp_attach(MlpState& s, Phys& P) {
  P.mlp_in_c = s.norm[0];
  P.mlp_in_s = s.norm[1];
  P.mlp_out_c = s.norm[2];
  P.mlp_out_s = s.norm[3];
  P.mlp_eps_lo = s.eps_lo;
  P.mlp_eps_hi = s.eps_hi;
}

// 1/theta of the state's internal energies with the handle's theta mode,
// written with a stride (in doubles) into the particle records.
inline void enqueue_theta_mlp(MlpState& s, hipStream_t st, const double* eps, double* invT,
                              int64_t stride, int64_t n, const Phys& P, uint32_t* status) {
  const int mode = s.trained ? P.theta_mode : 0;
  hipLaunchKernelGGL(k_theta<1>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, eps, invT,
                     stride, (int32_t*)nullptr, n, P, mlp_dev(s), mode, status);
}

inline void launch_theta(MlpState& s, hipStream_t st, const double* eps, double* theta,
                         int32_t* iters, int64_t n, const Phys& P, int mode) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_theta<0>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, eps, theta,
                     (int64_t)1, iters, n, P, mlp_dev(s), mode, (uint32_t*)nullptr);
}

inline int mlp_set(MlpState& s, const Phys& P, const float* w, const double* norm4,
                   std::string& err) {
  (void)P;
  if (mlp_ensure_weights(s)) { err = "allocation failed"; return DPDE_ENOMEM; }
  if (hipMemcpy(s.w, w, kNParam * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    err = "copy failed";
    return DPDE_EHIP;
  }
  hipLaunchKernelGGL(k_to_bf16, dim3((kNParam + 255) / 256), dim3(256), 0, nullptr, s.w, s.wb,
                     kNParam);
  if (hipDeviceSynchronize() != hipSuccess) { err = "conversion failed"; return DPDE_EHIP; }
  for (int k = 0; k < 4; ++k) s.norm[k] = norm4[k];
  // training range of eps implied by the normalisation: x in [-1, 1]
  s.eps_lo = std::exp(norm4[0] - norm4[1]);
  s.eps_hi = std::exp(norm4[0] + norm4[1]);
  s.trained = true;
  return DPDE_OK;
}

inline int mlp_get(MlpState& s, float* w, double* norm4, std::string& err) {
  if (!s.w) { err = "the surrogate has no weights"; return DPDE_EINVAL; }
  if (w && hipMemcpy(w, s.w, kNParam * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) {
    err = "copy failed";
    return DPDE_EHIP;
  }
  if (norm4)
    for (int k = 0; k < 4; ++k) norm4[k] = s.norm[k];
  return DPDE_OK;
}

inline int mlp_ensure_train_buffers(MlpState& s, int gblocks, int64_t loss_cap) {
  int rc;
  if (s.gblocks < gblocks) {
    if ((rc = mlp_alloc(s, &s.gpart, (size_t)gblocks * kNParam)) ||
        (rc = mlp_alloc(s, &s.lpart, gblocks)))
      return rc;
    s.gblocks = gblocks;
  }
  if (s.loss_cap < loss_cap) {
    if ((rc = mlp_alloc(s, &s.loss, loss_cap))) return rc;
    s.loss_cap = loss_cap;
  }
  return DPDE_OK;
}

inline int mlp_grad(MlpState& s, hipStream_t st, const float* x, const float* t, int64_t n,
                    float* loss, float* grad, std::string& err) {
  if (!s.w) { err = "the surrogate has no weights"; return DPDE_EINVAL; }
  if (n <= 0) { err = "n must be > 0"; return DPDE_EINVAL; }
  const int gb = (int)std::min<int64_t>(64, (n + kTrainThreads - 1) / kTrainThreads);
  if (mlp_ensure_train_buffers(s, gb, 1)) { err = "allocation failed"; return DPDE_ENOMEM; }
  hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3(gb), dim3(kTrainThreads), 0, st, (const float*)s.w, x, t,
                     n, (int64_t)0, n, 1.0f / (float)n, s.gpart, s.lpart);
  hipLaunchKernelGGL(k_mlp_reduce_adam, dim3(1), dim3(1024), 0, st, (const float*)s.gpart,
                     (const double*)s.lpart, gb, n, s.w, s.adam_m, s.adam_v, s.wb, 0.0f, 1.0f,
                     1.0f, 0, s.gsum, s.loss);
  if (hipMemcpyAsync(grad, s.gsum, kNParam * sizeof(float), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipMemcpyAsync(loss, s.loss, sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    err = "gradient kernels failed";
    return DPDE_EHIP;
  }
  return DPDE_OK;
}

inline int mlp_eval(MlpState& s, hipStream_t st, const float* x, float* y, int64_t n,
                    std::string& err) {
  if (!s.wb) { err = "the surrogate has no weights"; return DPDE_EINVAL; }
  if (n <= 0) return DPDE_OK;
  hipLaunchKernelGGL(k_mlp_eval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     (const float*)s.w, (const uint16_t*)s.wb, x, y, n);
  if (hipStreamSynchronize(st) != hipSuccess) { err = "inference kernel failed"; return DPDE_EHIP; }
  return DPDE_OK;
}

template <typename Cfg>
inline int mlp_train(MlpState& s, hipStream_t st, const Phys& P, const Cfg& cfg,
                     float* loss_curve, std::string& err) {
  if (!(cfg.theta_lo > 0 && cfg.theta_hi > cfg.theta_lo) || cfg.nsamples < 1 || cfg.iters < 0 ||
      cfg.batch < 1 || !(cfg.lr > 0)) {
    err = "bad training configuration";
    return DPDE_EINVAL;
  }
  if (mlp_ensure_weights(s)) { err = "allocation failed"; return DPDE_ENOMEM; }
  if (s.nsamp < cfg.nsamples) {
    if (mlp_alloc(s, &s.xs, cfg.nsamples) || mlp_alloc(s, &s.ts, cfg.nsamples)) {
      err = "allocation failed";
      return DPDE_ENOMEM;
    }
    s.nsamp = cfg.nsamples;
  }
  const double elo = eos_energy_host(P, cfg.theta_lo), ehi = eos_energy_host(P, cfg.theta_hi);
  s.norm[0] = 0.5 * (std::log(elo) + std::log(ehi));
  s.norm[1] = 0.5 * (std::log(ehi) - std::log(elo));
  s.norm[2] = 0.5 * (std::log(cfg.theta_lo) + std::log(cfg.theta_hi));
  s.norm[3] = 0.5 * (std::log(cfg.theta_hi) - std::log(cfg.theta_lo));
  s.eps_lo = elo;
  s.eps_hi = ehi;
  hipLaunchKernelGGL(k_mlp_samples, dim3((unsigned)((cfg.nsamples + 255) / 256)), dim3(256), 0, st,
                     (uint64_t)cfg.seed, (int64_t)cfg.nsamples, std::log(cfg.theta_lo),
                     std::log(cfg.theta_hi), P, s.norm[0], s.norm[1], s.norm[2], s.norm[3], s.xs,
                     s.ts);
  // initial weights: N(0, 1.5^2) input layer, N(0, 1) biases, N(0, 1/32) hidden
  std::vector<float> w0(kNParam);
  std::mt19937_64 gen(cfg.seed ^ 0x9E3779B97F4A7C15ull);
  std::normal_distribution<double> nd(0.0, 1.0);
  for (int k = 0; k < kNParam; ++k) {
    double sd;
    if (k < OFF_B1) sd = 1.5;
    else if (k < OFF_W2) sd = 1.0;
    else if (k < OFF_B2) sd = 1.0 / std::sqrt((double)kH);
    else if (k < OFF_W3) sd = 0.0;
    else if (k < OFF_B3) sd = 1.0 / std::sqrt((double)kH);
    else sd = 0.0;
    w0[k] = (float)(sd * nd(gen));
  }
  if (hipMemcpyAsync(s.w, w0.data(), kNParam * sizeof(float), hipMemcpyHostToDevice, st) !=
      hipSuccess) {
    err = "copy failed";
    return DPDE_EHIP;
  }
  (void)hipMemsetAsync(s.adam_m, 0, kNParam * sizeof(float), st);
  (void)hipMemsetAsync(s.adam_v, 0, kNParam * sizeof(float), st);
  hipLaunchKernelGGL(k_to_bf16, dim3((kNParam + 255) / 256), dim3(256), 0, st, (const float*)s.w,
                     s.wb, kNParam);
  const int gb = (int)std::min<int64_t>(64, (cfg.batch + kTrainThreads - 1) / kTrainThreads);
  if (mlp_ensure_train_buffers(s, gb, std::max<int64_t>(1, cfg.iters))) {
    err = "allocation failed";
    return DPDE_ENOMEM;
  }
  double b1p = 1.0, b2p = 1.0;
  for (int64_t it = 0; it < cfg.iters; ++it) {
    b1p *= 0.9;
    b2p *= 0.999;
    // cosine decay of the step size down to 1% of cfg.lr
    const double frac = cfg.iters > 1 ? (double)it / (double)(cfg.iters - 1) : 0.0;
    const double lr = cfg.lr * (0.01 + 0.99 * 0.5 * (1.0 + std::cos(M_PI * frac)));
    const int64_t begin = (it * (int64_t)cfg.batch) % cfg.nsamples;
    hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3(gb), dim3(kTrainThreads), 0, st, (const float*)s.w,
                       (const float*)s.xs, (const float*)s.ts, (int64_t)cfg.nsamples, begin,
                       (int64_t)cfg.batch, 1.0f / (float)cfg.batch, s.gpart, s.lpart);
    hipLaunchKernelGGL(k_mlp_reduce_adam, dim3(1), dim3(1024), 0, st, (const float*)s.gpart,
                       (const double*)s.lpart, gb, (int64_t)cfg.batch, s.w, s.adam_m, s.adam_v,
                       s.wb, (float)lr, (float)(1.0 - b1p), (float)(1.0 - b2p), 1,
                       (float*)nullptr, s.loss + it);
  }
  if (loss_curve && cfg.iters > 0 &&
      hipMemcpyAsync(loss_curve, s.loss, cfg.iters * sizeof(float), hipMemcpyDeviceToHost, st) !=
          hipSuccess) {
    err = "copy failed";
    return DPDE_EHIP;
  }
  if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) {
    err = "training kernels failed";
    return DPDE_EHIP;
  }
  s.trained = true;
  return DPDE_OK;
}

}  // namespace dpde
