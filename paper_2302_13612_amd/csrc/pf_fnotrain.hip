// Pointwise parts of the learned stepper for training (FP32, channel-first
// batches [B][channels][nvox]) and the optimiser:
//   lift        v_0 = P [f, c] + p
//   layer       u = W v + b + K v (K v from the spectral kernels), v' = GELU(u)
//   projection  z = Q_1 v + q_1, f~ = f + Q_2 GELU(z) + q_2
// with the backward of each (per-voxel chain rule), weight gradients as sums
// over batch and voxels of products of two channel fields (outer sums,
// per-chunk partials then a fixed-order reduction), and Adam.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/pf.h"

namespace pft2 {

constexpr int kMaxC = 64;    // channels of a layer (4, 8, 16, 32 or 64)
constexpr int kMaxH = 128;   // hidden units of the projection
constexpr int kNCond = 7;

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x) {
  return 0.5f * (1.f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * __expf(-0.5f * x * x);
}

int blocks(long n) {
  const long b = (n + 255) / 256;
  return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

// v0[b][c][i] = P[c][0] f[b][i] + sum_j P[c][1 + j] cond[b][j] + p[c]
__global__ __launch_bounds__(256) void k_lift(int B, int C, long nvox, const float* __restrict__ P,
                                              const float* __restrict__ p, const float* __restrict__ f,
                                              const float* __restrict__ cond, float* __restrict__ v0) {
  const long total = (long)B * nvox;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int b = (int)(t / nvox);
    const long i = t % nvox;
    const float e = f[t];
    for (int c = 0; c < C; ++c) {
      float k = p[c];
      for (int j = 0; j < kNCond; ++j) k += P[c * (1 + kNCond) + 1 + j] * cond[b * kNCond + j];
      v0[((long)b * C + c) * nvox + i] = P[c * (1 + kNCond)] * e + k;
    }
  }
}

// u = W v + bias + kv, vout = GELU(u)
template <int C>
__global__ __launch_bounds__(256) void k_layer_fwd(int B, long nvox, const float* __restrict__ W,
                                                   const float* __restrict__ bias, const float* __restrict__ v,
                                                   const float* __restrict__ kv, float* __restrict__ u,
                                                   float* __restrict__ vout) {
  __shared__ float sw[C * C];
  for (int j = threadIdx.x; j < C * C; j += blockDim.x) sw[j] = W[j];
  __syncthreads();
  const long total = (long)B * nvox;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int b = (int)(t / nvox);
    const long i = t % nvox;
    const float* vb = v + (long)b * C * nvox + i;
    float x[C];
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = vb[(long)c * nvox];
    for (int o = 0; o < C; ++o) {
      float a = bias[o];
#pragma unroll
      for (int c = 0; c < C; ++c) a += sw[o * C + c] * x[c];
      const long at = ((long)b * C + o) * nvox + i;
      a += kv[at];
      u[at] = a;
      vout[at] = gelu(a);
    }
  }
}

// z = Q1 v + q1 (stored), out = f + Q2 GELU(z) + q2
template <int C>
__global__ __launch_bounds__(256) void k_proj_fwd(int B, int H, long nvox, const float* __restrict__ Q1,
                                                  const float* __restrict__ q1, const float* __restrict__ Q2,
                                                  float q2, const float* __restrict__ v, const float* __restrict__ f,
                                                  float* __restrict__ z, float* __restrict__ out) {
  __shared__ float sq[kMaxH * C];
  for (int j = threadIdx.x; j < H * C; j += blockDim.x) sq[j] = Q1[j];
  __syncthreads();
  const long total = (long)B * nvox;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int b = (int)(t / nvox);
    const long i = t % nvox;
    const float* vb = v + (long)b * C * nvox + i;
    float x[C];
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = vb[(long)c * nvox];
    float acc = q2;
    for (int h = 0; h < H; ++h) {
      float a = q1[h];
#pragma unroll
      for (int c = 0; c < C; ++c) a += sq[h * C + c] * x[c];
      z[((long)b * H + h) * nvox + i] = a;
      acc += Q2[h] * gelu(a);
    }
    out[t] = f[t] + acc;
  }
}

// loss gradient g = scale (out - target); dz = g Q2 GELU'(z); hg = GELU(z);
// dv = Q1^T dz
template <int C>
__global__ __launch_bounds__(256) void k_proj_bwd(int B, int H, long nvox, const float* __restrict__ Q1,
                                                  const float* __restrict__ Q2, const float* __restrict__ z,
                                                  const float* __restrict__ out, const float* __restrict__ target,
                                                  float scale, float* __restrict__ g, float* __restrict__ dz,
                                                  float* __restrict__ hg, float* __restrict__ dv) {
  __shared__ float sq[kMaxH * C];
  for (int j = threadIdx.x; j < H * C; j += blockDim.x) sq[j] = Q1[j];
  __syncthreads();
  const long total = (long)B * nvox;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int b = (int)(t / nvox);
    const long i = t % nvox;
    const float gv = scale * (out[t] - target[t]);
    g[t] = gv;
    float d[C];
#pragma unroll
    for (int c = 0; c < C; ++c) d[c] = 0.f;
    for (int h = 0; h < H; ++h) {
      const long at = ((long)b * H + h) * nvox + i;
      const float zz = z[at];
      const float dzh = gv * Q2[h] * gelu_d(zz);
      dz[at] = dzh;
      hg[at] = gelu(zz);
#pragma unroll
      for (int c = 0; c < C; ++c) d[c] += sq[h * C + c] * dzh;
    }
#pragma unroll
    for (int c = 0; c < C; ++c) dv[((long)b * C + c) * nvox + i] = d[c];
  }
}

// du = dvout GELU'(u)
__global__ __launch_bounds__(256) void k_gelu_bwd(long n, const float* __restrict__ dvout, const float* __restrict__ u,
                                                  float* __restrict__ du) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
    du[t] = dvout[t] * gelu_d(u[t]);
}

// dv = W^T du + dvs
template <int C>
__global__ __launch_bounds__(256) void k_layer_bwd(int B, long nvox, const float* __restrict__ W,
                                                   const float* __restrict__ du, const float* __restrict__ dvs,
                                                   float* __restrict__ dv) {
  __shared__ float sw[C * C];
  for (int j = threadIdx.x; j < C * C; j += blockDim.x) sw[j] = W[j];
  __syncthreads();
  const long total = (long)B * nvox;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int b = (int)(t / nvox);
    const long i = t % nvox;
    float d[C];
#pragma unroll
    for (int c = 0; c < C; ++c) d[c] = 0.f;
    for (int o = 0; o < C; ++o) {
      const float x = du[((long)b * C + o) * nvox + i];
#pragma unroll
      for (int c = 0; c < C; ++c) d[c] += sw[o * C + c] * x;
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const long at = ((long)b * C + c) * nvox + i;
      dv[at] = d[c] + dvs[at];
    }
  }
}

// Outer sums out[a][c] = sum_{b, i} X[b][a][i] Y[b][c][i] (Y null: 1), over
// voxel chunks: block (chunk, a-tile of 16, c-tile of 16) writes its 16 x 16
// partial for its chunk; k_reduce then adds the chunks in order.
constexpr int kTile = 16;
constexpr long kChunk = 4096;

__global__ __launch_bounds__(256) void k_outer_part(int B, int MA, int MC, long nvox, const float* __restrict__ X,
                                                    const float* __restrict__ Y, float* __restrict__ part) {
  const long nchunk = (nvox + kChunk - 1) / kChunk;
  const int ta = blockIdx.y, tc = blockIdx.z;
  const long ch = blockIdx.x % nchunk;
  const int b = (int)(blockIdx.x / nchunk);
  const int a = ta * kTile + threadIdx.x / kTile, c = tc * kTile + threadIdx.x % kTile;
  __shared__ float xs[kTile][65], ys[kTile][65];  // padded: rows fall in different banks
  float acc = 0.f;
  const long i0 = ch * kChunk, i1 = (i0 + kChunk < nvox) ? i0 + kChunk : nvox;
  for (long s = i0; s < i1; s += 64) {
    for (int j = threadIdx.x; j < kTile * 64; j += blockDim.x) {
      const int r = j / 64, k = j % 64;
      const long i = s + k;
      const int aa = ta * kTile + r, cc = tc * kTile + r;
      xs[r][k] = (i < i1 && aa < MA) ? X[((long)b * MA + aa) * nvox + i] : 0.f;
      ys[r][k] = (i < i1 && cc < MC) ? (Y ? Y[((long)b * MC + cc) * nvox + i] : 1.f) : 0.f;
    }
    __syncthreads();
    const int ra = threadIdx.x / kTile, rc = threadIdx.x % kTile;
    for (int k = 0; k < 64; ++k) acc += xs[ra][k] * ys[rc][k];
    __syncthreads();
  }
  const long nblk = (long)B * nchunk;
  if (a < MA && c < MC) part[((long)a * MC + c) * nblk + blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_reduce(long nout, long nblk, const float* __restrict__ part,
                                                float* __restrict__ out, int accumulate) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < nout; t += (long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (long k = 0; k < nblk; ++k) s += part[t * nblk + k];
    out[t] = accumulate ? out[t] + (float)s : (float)s;
  }
}

// dP[c][1 + j] = sum_b dK[b][c] cond[b][j], dp[c] = sum_b dK[b][c] (dK: per-sample
// channel sums of the lift's output gradient)
__global__ void k_cond_grad(int B, int C, const float* __restrict__ dK, const float* __restrict__ cond,
                            float* __restrict__ dP, float* __restrict__ dp) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += dK[b * C + c];
  dp[c] = s;
  for (int j = 0; j < kNCond; ++j) {
    float a = 0.f;
    for (int b = 0; b < B; ++b) a += dK[b * C + c] * cond[b * kNCond + j];
    dP[c * (1 + kNCond) + 1 + j] = a;
  }
}

// Adam with bias correction (step t >= 1)
__global__ __launch_bounds__(256) void k_adam(long n, float* __restrict__ w, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                              float b2, float eps, float c1, float c2) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.f - b1) * gt;
    const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    w[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
  }
}

hipError_t done() { return hipGetLastError(); }

// Per-chunk partials of the outer sums for callers that cannot allocate: a
// fixed array of the library, 16 MiB on every GPU it runs on, held until the
// process ends. Host code never uses the array's name as an address: its
// device address is taken once per device (hipGetSymbolAddress, with that
// device current) and kept in scratch_dev.
constexpr size_t kScratchFloats = (size_t)4 << 20;
static __device__ __align__(256) float scratch[kScratchFloats];
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
float* scratch_dev[kMaxDevices] = {};

// Device address of this library's scratch array on the device of stream s
// (NULL: the current device).
int scratch_of(hipStream_t s, float** out) {
  int dev = 0;
  hipError_t e = s ? hipStreamGetDevice(s, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) return PF_EDEVICE;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return PF_EDEVICE;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return PF_EDEVICE;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) hipSetDevice(cur);
    if (e != hipSuccess || !p) return PF_EDEVICE;
    scratch_dev[dev] = static_cast<float*>(p);
  }
  *out = scratch_dev[dev];
  return PF_OK;
}

#define PF_SWITCH_C(c, BODY)                                     \
  switch (c) {                                                    \
    case 4: { constexpr int CC = 4; BODY; } break;                \
    case 8: { constexpr int CC = 8; BODY; } break;                \
    case 16: { constexpr int CC = 16; BODY; } break;              \
    case 32: { constexpr int CC = 32; BODY; } break;              \
    case 64: { constexpr int CC = 64; BODY; } break;              \
    default: return PF_EINVAL;                                    \
  }

}  // namespace pft2

using namespace pft2;

extern "C" {

int pf_nt_lift(int32_t B, int32_t C, int64_t nvox, const float* P, const float* p, const float* f,
               const float* cond, float* v0, void* stream) {
  if (B < 1 || C < 1 || C > kMaxC || nvox < 1 || !P || !p || !f || !cond || !v0) return PF_EINVAL;
  k_lift<<<blocks(B * nvox), 256, 0, (hipStream_t)stream>>>(B, C, nvox, P, p, f, cond, v0);
  return done() == hipSuccess ? PF_OK : PF_EDEVICE;
}

int pf_nt_layer_forward(int32_t B, int32_t C, int64_t nvox, const float* W, const float* bias, const float* v,
                        const float* kv, float* u, float* vout, void* stream) {
  if (B < 1 || C < 1 || C > kMaxC || nvox < 1 || !W || !bias || !v || !kv || !u || !vout) return PF_EINVAL;
  PF_SWITCH_C(C, (k_layer_fwd<CC><<<blocks(B * nvox), 256, 0, (hipStream_t)stream>>>(B, nvox, W, bias, v, kv, u, vout)));
  return done() == hipSuccess ? PF_OK : PF_EDEVICE;
}

int pf_nt_project_forward(int32_t B, int32_t C, int32_t H, int64_t nvox, const float* Q1, const float* q1,
                          const float* Q2, float q2, const float* v, const float* f, float* z, float* out,
                          void* stream) {
  if (B < 1 || C < 1 || C > kMaxC || H < 1 || H > kMaxH || nvox < 1 || !Q1 || !q1 || !Q2 || !v || !f || !z || !out)
    return PF_EINVAL;
  PF_SWITCH_C(C, (k_proj_fwd<CC><<<blocks(B * nvox), 256, 0, (hipStream_t)stream>>>(B, H, nvox, Q1, q1, Q2, q2, v, f, z, out)));
  return done() == hipSuccess ? PF_OK : PF_EDEVICE;
}

int pf_nt_project_backward(int32_t B, int32_t C, int32_t H, int64_t nvox, const float* Q1, const float* Q2,
                           const float* z, const float* out, const float* target, float scale, float* g, float* dz,
                           float* hg, float* dv, void* stream) {
  if (B < 1 || C < 1 || C > kMaxC || H < 1 || H > kMaxH || nvox < 1 || !Q1 || !Q2 || !z || !out || !target || !g ||
      !dz || !hg || !dv)
    return PF_EINVAL;
  PF_SWITCH_C(C, (k_proj_bwd<CC><<<blocks(B * nvox), 256, 0, (hipStream_t)stream>>>(B, H, nvox, Q1, Q2, z, out,
                                                                                    target, scale, g, dz, hg, dv)));
  return done() == hipSuccess ? PF_OK : PF_EDEVICE;
}

int pf_nt_gelu_backward(int64_t n, const float* dvout, const float* u, float* du, void* stream) {
  if (n < 1 || !dvout || !u || !du) return PF_EINVAL;
  k_gelu_bwd<<<blocks(n), 256, 0, (hipStream_t)stream>>>(n, dvout, u, du);
  return done() == hipSuccess ? PF_OK : PF_EDEVICE;
}

int pf_nt_layer_input_grad(int32_t B, int32_t C, int64_t nvox, const float* W, const float* du, const float* dvs,
                           float* dv, void* stream) {
  if (B < 1 || C < 1 || C > kMaxC || nvox < 1 || !W || !du || !dvs || !dv) return PF_EINVAL;
  PF_SWITCH_C(C, (k_layer_bwd<CC><<<blocks(B * nvox), 256, 0, (hipStream_t)stream>>>(B, nvox, W, du, dvs, dv)));
  return done() == hipSuccess ? PF_OK : PF_EDEVICE;
}

int pf_nt_outer_workspace(int32_t B, int32_t MA, int32_t MC, int64_t nvox, size_t* bytes) {
  if (!bytes || B < 1 || MA < 1 || MC < 1 || nvox < 1) return PF_EINVAL;
  const long nchunk = (long)((nvox + kChunk - 1) / kChunk);
  *bytes = sizeof(float) * (size_t)MA * MC * B * nchunk;
  return PF_OK;
}

int pf_nt_outer_sum(int32_t B, int32_t MA, int32_t MC, int64_t nvox, const float* X, const float* Y, float* out,
                    int32_t accumulate, float* work, size_t work_bytes, void* stream) {
  size_t need = 0;
  if (pf_nt_outer_workspace(B, MA, MC, nvox, &need) != PF_OK || !X || !out || !work) return PF_EINVAL;
  if (work_bytes < need) return PF_ENOMEM;
  const long nchunk = (long)((nvox + kChunk - 1) / kChunk);
  const dim3 grid((unsigned)(B * nchunk), (unsigned)((MA + kTile - 1) / kTile), (unsigned)((MC + kTile - 1) / kTile));
  hipStream_t s = (hipStream_t)stream;
  k_outer_part<<<grid, kTile * kTile, 0, s>>>(B, MA, MC, nvox, X, Y, work);
  k_reduce<<<blocks((long)MA * MC), 256, 0, s>>>((long)MA * MC, (long)B * nchunk, work, out, accumulate);
  return done() == hipSuccess ? PF_OK : PF_EDEVICE;
}

int pf_nt_outer_sum_noalloc(int32_t B, int32_t MA, int32_t MC, int64_t nvox, const float* X, const float* Y,
                            float* out, int32_t accumulate, void* stream) {
  size_t need = 0;
  if (pf_nt_outer_workspace(B, MA, MC, nvox, &need) != PF_OK || !X || !out) return PF_EINVAL;
  if (need > sizeof(float) * kScratchFloats) return PF_ENOMEM;
  float* work = nullptr;
  hipStream_t s = (hipStream_t)stream;
  const int rc = scratch_of(s, &work);
  if (rc != PF_OK) return rc;
  // every partial is written before k_reduce reads it: nothing to clear
  const long nchunk = (long)((nvox + kChunk - 1) / kChunk);
  const dim3 grid((unsigned)(B * nchunk), (unsigned)((MA + kTile - 1) / kTile), (unsigned)((MC + kTile - 1) / kTile));
  k_outer_part<<<grid, kTile * kTile, 0, s>>>(B, MA, MC, nvox, X, Y, work);
  k_reduce<<<blocks((long)MA * MC), 256, 0, s>>>((long)MA * MC, (long)B * nchunk, work, out, accumulate);
  return done() == hipSuccess ? PF_OK : PF_EDEVICE;
}

int pf_nt_cond_grad(int32_t B, int32_t C, const float* dK, const float* cond, float* dP, float* dp, void* stream) {
  if (B < 1 || C < 1 || !dK || !cond || !dP || !dp) return PF_EINVAL;
  k_cond_grad<<<(C + 63) / 64, 64, 0, (hipStream_t)stream>>>(B, C, dK, cond, dP, dp);
  return done() == hipSuccess ? PF_OK : PF_EDEVICE;
}

int pf_nt_adam(int64_t n, float* w, const float* g, float* m, float* v, float lr, float beta1, float beta2, float eps,
               int32_t step, void* stream) {
  if (n < 1 || !w || !g || !m || !v || step < 1) return PF_EINVAL;
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  k_adam<<<blocks(n), 256, 0, (hipStream_t)stream>>>(n, w, g, m, v, lr, beta1, beta2, eps, c1, c2);
  return done() == hipSuccess ? PF_OK : PF_EDEVICE;
}

}  // extern "C"
