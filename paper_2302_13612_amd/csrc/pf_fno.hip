// Fourier-neural-operator macro stepper (gfx950): forward pass of
//   v_0 = P [f, c] + p,  v_l = GELU(W_l v + b_l + K_l v) (l = 1..4),
//   f~ = f + Q_2 GELU(Q_1 v_4 + q_1) + q_2,
// with K v the inverse real transform of R(k) times the transform of v on the
// kept modes (kx < m, ky and kz in [0, m) u [n - m, n)).
//
// Only 12 x 24 x 24 of the modes are kept, so the transforms are truncated
// discrete Fourier sums, not FFTs: x (full real rows -> m complex), y and z
// (full length -> 2m kept), channel mixing per kept mode, and the inverses.
// The full-resolution work is the x sums and the pointwise channel mixing;
// the mixing (32 x 32 per voxel) and the projection's first layer (32 -> 128
// per voxel) run on the matrix cores as BF16 MFMA with FP32 accumulation.
//
// Layouts: activations v [z][y][x][C] BF16 (C = 32, channel-last);
// transforms X [z][y or ky'][kx][re/im][C] FP32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pf_fno.hpp"

namespace pfn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }

// Signed kept index -> frequency on an axis of length n.
__device__ __forceinline__ int kept_freq(int kk, int m, int n) { return kk < m ? kk : n - 2 * m + kk; }

// ---------------------------------------------------------------- lift
// v_0[vox][c] = P0[c] f + K[c] (K folds the constant conditioning channels).
__global__ __launch_bounds__(256) void k_lift(const FArgs a, const float* __restrict__ eta,
                                              uint16_t* __restrict__ v) {
  const float* coef = a.lift;
  const size_t vox = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (vox >= a.nvox) return;
  const float f = eta[vox];
  uint4* dst = reinterpret_cast<uint4*>(v + vox * kC);
#pragma unroll
  for (int q = 0; q < kC / 8; ++q) {
    uint32_t w[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int c = 8 * q + 2 * h;
      const uint16_t lo = f2bf(coef[c] * f + coef[kC + c]);
      const uint16_t hi = f2bf(coef[c + 1] * f + coef[kC + c + 1]);
      w[h] = (uint32_t)lo | ((uint32_t)hi << 16);
    }
    dst[q] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

// ------------------------------------------------------- x forward sums
// X1[row][kx][ri][c] = sum_x v[row][x][c] e^{-2 pi i kx x / nx}, kx < m.
// One block per row; the row is staged in LDS as FP32.
__global__ __launch_bounds__(256) void k_xdft(const FArgs a, const uint16_t* __restrict__ v) {
  extern __shared__ float sm[];
  float* row = sm;                       // [nx][C]
  float2* tw = reinterpret_cast<float2*>(sm + a.nx * kC);  // [nx]
  const int r = blockIdx.x;
  const uint4* src = reinterpret_cast<const uint4*>(v + (size_t)r * a.nx * kC);
  for (int i = threadIdx.x; i < a.nx * kC / 8; i += 256) {
    const uint4 q = src[i];
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      row[8 * i + 2 * h] = bf2f((uint16_t)(w[h] & 0xffffu));
      row[8 * i + 2 * h + 1] = bf2f((uint16_t)(w[h] >> 16));
    }
  }
  for (int i = threadIdx.x; i < a.nx; i += 256) tw[i] = a.twx[i];
  __syncthreads();
  const int c = threadIdx.x % kC, g = threadIdx.x / kC;
  float* out = a.X1 + (size_t)r * a.m * 2 * kC;
  for (int kx = g; kx < a.m; kx += 8) {
    float re = 0.f, im = 0.f;
    int j = 0;
    for (int x = 0; x < a.nx; ++x) {
      const float val = row[x * kC + c];
      const float2 w = tw[j];
      re += val * w.x;
      im += val * w.y;
      j += kx;
      if (j >= a.nx) j -= a.nx;
    }
    out[(kx * 2) * kC + c] = re;
    out[(kx * 2 + 1) * kC + c] = im;
  }
}

// ---------------------------------------------------- y and z sums
// Complex sums along an axis of a [..][n][m][2][C] array for one (outer, kx):
// forward: out[kk] = sum_t in[t] e^{-2 pi i k(kk) t / n} over the 2m kept k;
// inverse: out[t] = sum_kk in[kk] e^{+2 pi i k(kk) t / n}.
// One block per (outer, kx); the input column is staged in LDS.
template <bool FWD>
__global__ __launch_bounds__(256) void k_ysum(const FArgs a, const float* __restrict__ in, float* __restrict__ out) {
  extern __shared__ float sm[];
  const int ny = a.ny, m = a.m, my = 2 * m;
  const int nin = FWD ? ny : my, nout = FWD ? my : ny;
  float* col = sm;                                        // [nin][2][C]
  float2* tw = reinterpret_cast<float2*>(sm + nin * 2 * kC);  // [ny]
  const int z = blockIdx.x / m, kx = blockIdx.x % m;
  const size_t in_base = (size_t)z * nin * m * 2 * kC + (size_t)kx * 2 * kC;
  const size_t out_base = (size_t)z * nout * m * 2 * kC + (size_t)kx * 2 * kC;
  for (int i = threadIdx.x; i < nin * 2 * kC; i += 256) {
    const int t = i / (2 * kC), e = i % (2 * kC);
    col[i] = in[in_base + (size_t)t * m * 2 * kC + e];
  }
  for (int i = threadIdx.x; i < ny; i += 256) tw[i] = a.twy[i];
  __syncthreads();
  const int c = threadIdx.x % kC, g = threadIdx.x / kC;
  for (int o = g; o < nout; o += 8) {
    float re = 0.f, im = 0.f;
    if (FWD) {
      const int k = kept_freq(o, m, ny);
      int j = 0;
      for (int t = 0; t < ny; ++t) {
        const float xr = col[(2 * t) * kC + c], xi = col[(2 * t + 1) * kC + c];
        const float2 w = tw[j];  // e^{-2 pi i j / ny}
        re += xr * w.x - xi * w.y;
        im += xr * w.y + xi * w.x;
        j += k;
        if (j >= ny) j -= ny;
      }
    } else {
      for (int kk = 0; kk < my; ++kk) {
        const int k = kept_freq(kk, m, ny);
        const int j = (int)(((long)k * o) % ny);
        const float2 w = tw[j];  // conjugate for the inverse
        const float xr = col[(2 * kk) * kC + c], xi = col[(2 * kk + 1) * kC + c];
        re += xr * w.x + xi * w.y;
        im += xi * w.x - xr * w.y;
      }
    }
    out[out_base + (size_t)o * m * 2 * kC + c] = re;
    out[out_base + (size_t)o * m * 2 * kC + kC + c] = im;
  }
}

// z pass: one block per kept (ky', kx): forward z sums to the 2m kept kz,
// channel mixing by R(kz', ky', kx) (complex, C x C, BF16), inverse z sums.
__global__ __launch_bounds__(256) void k_zmix(const FArgs a, const uint16_t* __restrict__ R) {
  extern __shared__ float sm[];
  const int nz = a.nz, m = a.m, my = 2 * m;
  float* col = sm;                                // [nz][2][C]
  float* zs = col + nz * 2 * kC;                  // [2m][2][C]
  float* os = zs + my * 2 * kC;                   // [2m][2][C]
  float2* tw = reinterpret_cast<float2*>(os + my * 2 * kC);  // [nz]
  const int kyy = blockIdx.x / m, kx = blockIdx.x % m;
  const size_t zstride = (size_t)my * m * 2 * kC;
  const size_t base = (size_t)kyy * m * 2 * kC + (size_t)kx * 2 * kC;
  for (int i = threadIdx.x; i < nz * 2 * kC; i += 256) {
    const int t = i / (2 * kC), e = i % (2 * kC);
    col[i] = a.X2[base + (size_t)t * zstride + e];
  }
  for (int i = threadIdx.x; i < nz; i += 256) tw[i] = a.twz[i];
  __syncthreads();
  const int c = threadIdx.x % kC, g = threadIdx.x / kC;
  for (int kk = g; kk < my; kk += 8) {
    const int k = kept_freq(kk, m, nz);
    float re = 0.f, im = 0.f;
    int j = 0;
    for (int t = 0; t < nz; ++t) {
      const float xr = col[(2 * t) * kC + c], xi = col[(2 * t + 1) * kC + c];
      const float2 w = tw[j];
      re += xr * w.x - xi * w.y;
      im += xr * w.y + xi * w.x;
      j += k;
      if (j >= nz) j -= nz;
    }
    zs[(2 * kk) * kC + c] = re;
    zs[(2 * kk + 1) * kC + c] = im;
  }
  __syncthreads();
  // mixing: os[kz'][o] = sum_i R[kz'][ky'][kx][o][i] zs[kz'][i]
  for (int kk = g; kk < my; kk += 8) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(
        R + ((((size_t)kk * my + kyy) * m + kx) * kC + c) * kC * 2);
    float re = 0.f, im = 0.f;
#pragma unroll 8
    for (int i = 0; i < kC; ++i) {
      const uint32_t p = w[i];
      const float rr = bf2f((uint16_t)(p & 0xffffu)), ri = bf2f((uint16_t)(p >> 16));
      const float xr = zs[(2 * kk) * kC + i], xi = zs[(2 * kk + 1) * kC + i];
      re += rr * xr - ri * xi;
      im += rr * xi + ri * xr;
    }
    os[(2 * kk) * kC + c] = re;
    os[(2 * kk + 1) * kC + c] = im;
  }
  __syncthreads();
  for (int t = g; t < nz; t += 8) {
    float re = 0.f, im = 0.f;
    for (int kk = 0; kk < my; ++kk) {
      const int k = kept_freq(kk, m, nz);
      const float2 w = tw[(int)(((long)k * t) % nz)];
      const float xr = os[(2 * kk) * kC + c], xi = os[(2 * kk + 1) * kC + c];
      re += xr * w.x + xi * w.y;
      im += xi * w.x - xr * w.y;
    }
    a.Y2[base + (size_t)t * zstride + c] = re;
    a.Y2[base + (size_t)t * zstride + kC + c] = im;
  }
}

// ------------------------------------------------ matrix-core helpers
// v_mfma_f32_32x32x16_bf16: lane l supplies A[l % 32][8 (l / 32) + 0..7] and
// B[8 (l / 32) + 0..7][l % 32]; it receives D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]
// in accumulator r.
__device__ __forceinline__ int mfma_row(int r, int lane) { return 8 * (r / 4) + 4 * (lane / 32) + (r % 4); }

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
  const uint4 q = *reinterpret_cast<const uint4*>(p);
  bf16x8 out;
  __builtin_memcpy(&out, &q, 16);
  return out;
}

// D (32 voxels x 32 outputs) = v[x0 .. x0+31][0..31] . Wt where Wt[i][o] = Wm[o][i]
__device__ __forceinline__ f32x16 mix32(const uint16_t* __restrict__ vrow, int x0, const uint16_t* __restrict__ Wm,
                                        int lane) {
  const int i = lane % 32, kb = 8 * (lane / 32);
  f32x16 acc = {};
  const uint16_t* ap = vrow + (size_t)(x0 + i) * kC + kb;
  const uint16_t* bp = Wm + (size_t)i * kC + kb;
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load8(ap), load8(bp), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load8(ap + 16), load8(bp + 16), acc, 0, 0, 0);
  return acc;
}

// ------------------------------------------- x inverse + local mixing
// v'[x][o] = GELU(sum_i W[o][i] v[x][i] + b[o]
//                 + s sum_kx w_kx Re(Y1[kx][o] e^{2 pi i kx x / nx})),
// s = 1 / (nx ny nz), w = 1 (kx = 0) or 2. One block per row, one wave per
// 32 voxels.
__global__ __launch_bounds__(256) void k_xinv_mix(const FArgs a, const uint16_t* __restrict__ vin,
                                                  uint16_t* __restrict__ vout, const uint16_t* __restrict__ Wm,
                                                  const float* __restrict__ bias) {
  extern __shared__ float sm[];
  float* y1 = sm;                                        // [m][2][C]
  float2* tw = reinterpret_cast<float2*>(sm + a.m * 2 * kC);  // [nx]
  const int r = blockIdx.x;
  const float* ysrc = a.Y1 + (size_t)r * a.m * 2 * kC;
  for (int i = threadIdx.x; i < a.m * 2 * kC; i += blockDim.x) y1[i] = ysrc[i];
  for (int i = threadIdx.x; i < a.nx; i += blockDim.x) tw[i] = a.twx[i];
  __syncthreads();
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64, nwave = blockDim.x / 64;
  const int o = lane % 32;
  const float bo = bias[o];
  const uint16_t* vrow = vin + (size_t)r * a.nx * kC;
  uint16_t* orow = vout + (size_t)r * a.nx * kC;
  for (int x0 = 32 * wave; x0 < a.nx; x0 += 32 * nwave) {
    const f32x16 acc = mix32(vrow, x0, Wm, lane);
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      const int x = x0 + mfma_row(rr, lane);
      float sp = 0.f;
      int j = 0;
      for (int kx = 0; kx < a.m; ++kx) {
        const float2 w = tw[j];  // e^{-2 pi i kx x / nx}; inverse uses the conjugate
        const float yr = y1[(2 * kx) * kC + o], yi = y1[(2 * kx + 1) * kC + o];
        const float re = yr * w.x + yi * w.y;
        sp += (kx == 0 ? 1.f : 2.f) * re;
        j += x;
        if (j >= a.nx) j -= a.nx;
      }
      orow[(size_t)x * kC + o] = f2bf(gelu(acc[rr] + bo + a.inv_ntot * sp));
    }
  }
}

// ------------------------------------------------------- projection
// f~[x] = f[x] + sum_h Q2[h] GELU(sum_i Q1[h][i] v[x][i] + q1[h]) + q2.
__global__ __launch_bounds__(256) void k_proj(const FArgs a, const uint16_t* __restrict__ v,
                                              const float* __restrict__ eta, float* __restrict__ out) {
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const size_t tile = (size_t)blockIdx.x * 4 + wave;   // 32 voxels per wave
  const size_t x0 = tile * 32;
  if (x0 >= a.nvox) return;
  float part[16];
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) part[rr] = 0.f;
  const uint16_t* vt = v + x0 * kC;
  for (int h0 = 0; h0 < kH; h0 += 32) {
    const f32x16 acc = mix32(vt, 0, a.Q1 + (size_t)h0 * kC, lane);
    const int h = h0 + lane % 32;
    const float qb = a.q1[h], q2w = a.Q2[h];
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) part[rr] += q2w * gelu(acc[rr] + qb);
  }
  // sum over the 32 hidden units held by lanes of the same half-wave
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) {
    float s = part[rr];
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    part[rr] = s;
  }
  if (lane % 32 == 0) {
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      const size_t x = x0 + mfma_row(rr, lane);
      out[x] = eta[x] + part[rr] + a.q2;
    }
  }
}

}  // namespace pfn

// ====================================================================== host
namespace pfn {

size_t lds_xdft(const FArgs& a) { return (size_t)a.nx * kC * 4 + (size_t)a.nx * 8; }
size_t lds_ysum(const FArgs& a, bool fwd) {
  return (size_t)(fwd ? a.ny : 2 * a.m) * 2 * kC * 4 + (size_t)a.ny * 8;
}
size_t lds_zmix(const FArgs& a) { return ((size_t)a.nz + 4 * a.m) * 2 * kC * 4 + (size_t)a.nz * 8; }
size_t lds_xinv(const FArgs& a) { return (size_t)a.m * 2 * kC * 4 + (size_t)a.nx * 8; }

hipError_t forward(const FArgs& a, const float* eta_in, float* eta_out, hipStream_t s) {
  const int rows = a.nz * a.ny;
  k_lift<<<(unsigned)((a.nvox + 255) / 256), 256, 0, s>>>(a, eta_in, a.va);
  uint16_t* vin = a.va;
  uint16_t* vout = a.vb;
  for (int l = 0; l < kLayers; ++l) {
    k_xdft<<<rows, 256, lds_xdft(a), s>>>(a, vin);
    k_ysum<true><<<a.nz * a.m, 256, lds_ysum(a, true), s>>>(a, a.X1, a.X2);
    k_zmix<<<2 * a.m * a.m, 256, lds_zmix(a), s>>>(a, a.R + (size_t)l * a.r_stride);
    k_ysum<false><<<a.nz * a.m, 256, lds_ysum(a, false), s>>>(a, a.Y2, a.Y1);
    k_xinv_mix<<<rows, 256, lds_xinv(a), s>>>(a, vin, vout, a.W + (size_t)l * kC * kC, a.b + (size_t)l * kC);
    uint16_t* t = vin;
    vin = vout;
    vout = t;
  }
  k_proj<<<(unsigned)((a.nvox / 32 + 3) / 4), 256, 0, s>>>(a, vin, eta_in, eta_out);
  return hipGetLastError();
}

}  // namespace pfn
