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
// both x sums (2m x nx twiddles against the 32 channels of a row), the mixing
// (32 x 32 per voxel) and the projection's first layer (32 -> 128 per voxel)
// run on the matrix cores as BF16 MFMA with FP32 accumulation, FP32 operands
// (twiddles, transformed rows) entering as BF16 hi and lo parts.
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

// erf by Abramowitz & Stegun, Handbook of Mathematical Functions, formula
// 7.1.26 (after Hastings): erf(x) = 1 - t (a1 + t (a2 + ... + t a5)) e^{-x^2},
// t = 1 / (1 + p x) for x >= 0, odd for x < 0; absolute error <= 1.5e-7 in
// exact arithmetic, 4.7e-7 as evaluated here in FP32 (GELU: 4.6e-7), far
// below the BF16 rounding of the activations. One hardware reciprocal and one
// hardware exp2 in place of the library's two-range erf (about half the
// instructions), which matters where 128 of them are taken per voxel.
__device__ __forceinline__ float erf_as(float x) {
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.f));
  float q = fmaf(t, 1.061405429f, -1.453152027f);
  q = fmaf(t, q, 1.421413741f);
  q = fmaf(t, q, -0.284496736f);
  q = fmaf(t, q, 0.254829592f);
  const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * ax * ax);
  return copysignf(fmaf(-t * q, e, 1.f), x);
}

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.f + erf_as(x * 0.70710678118654752f)); }

// Signed kept index -> frequency on an axis of length n.
__device__ __forceinline__ int kept_freq(int kk, int m, int n) { return kk < m ? kk : n - 2 * m + kk; }

// Inverse sums step the twiddle index k(kk) t mod n by t (< n) along the kept
// list: from 0 for kk < m, and from (n - m) t mod n = (-m t) mod n for the
// negative frequencies kk >= m.
__device__ __forceinline__ int inv_start(int m, int t, int n) {
  const int r = (m * t) % n;
  return r == 0 ? 0 : n - r;
}

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

// D (32 outputs x 32 voxels) = Wm . v[x0 .. x0+31][0..31]^T: accumulator r of
// lane l holds output o = mfma_row(r, l) of voxel x0 + l % 32, so a lane owns
// four runs of four consecutive outputs of one voxel (stored as 8 bytes each).
__device__ __forceinline__ f32x16 mix32(const uint16_t* __restrict__ vrow, int x0, const uint16_t* __restrict__ Wm,
                                        int lane) {
  const int i = lane % 32, kb = 8 * (lane / 32);
  f32x16 acc = {};
  const uint16_t* wp = Wm + (size_t)i * kC + kb;
  const uint16_t* vp = vrow + (size_t)(x0 + i) * kC + kb;
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load8(wp), load8(vp), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load8(wp + 16), load8(vp + 16), acc, 0, 0, 0);
  return acc;
}

// ------------------------------------------------------- x forward sums
// X1[row][j][c] = sum_x WF[j][x] v[row][x][c], j = 2 kx + (re, im), kx < m,
// with WF[2 kx][x] = cos(2 pi kx x / nx), WF[2 kx + 1][x] = -sin(2 pi kx x / nx)
// and rows j >= 2m zero. On the matrix cores: A = WF (32 j by 16 x per
// product, as the BF16 hi and lo parts of the FP32 twiddle), B = the row's
// activations. The channel-last row is transposed to [c][x] in the wave's LDS
// so each lane reads its eight consecutive x of one channel in one 16-byte
// load. Four waves take one row each per round; the twiddles sit in LDS.
constexpr int kDftRounds = 4;  // rounds of four rows per block

__device__ __forceinline__ int xpitch(int nx) { return nx + 8; }  // bf16 per LDS row, a 16-byte multiple

__global__ __launch_bounds__(256) void k_xdft(const FArgs a, const uint16_t* __restrict__ v) {
  extern __shared__ __align__(16) uint16_t xs[];
  const int nx = a.nx, pitch = xpitch(nx), pdw = pitch / 2;
  uint16_t* wf = xs;                    // [hi, lo][32][pitch]
  uint16_t* tr = xs + 2 * 32 * pitch;   // [wave][32][pitch]
  const int n8 = nx / 8;
  for (int i = threadIdx.x; i < 2 * 32 * n8; i += 256) {
    const int hj = i / n8, x8 = i % n8;  // hj = h * 32 + j
    *reinterpret_cast<uint4*>(wf + hj * pitch + 8 * x8) =
        *reinterpret_cast<const uint4*>(a.wxf + (size_t)hj * nx + 8 * x8);
  }
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int i = lane % 32, kb = 8 * (lane / 32);
  uint16_t* t = tr + wave * 32 * pitch;
  uint32_t* tdw = reinterpret_cast<uint32_t*>(t);
  const int rows = a.ny * a.nz, m2 = 2 * a.m;
  for (int k = 0; k < kDftRounds; ++k) {
    const int row = (blockIdx.x * kDftRounds + k) * 4 + wave;
    const bool active = row < rows;
    __syncthreads();  // the twiddles are in place; the previous round's reads are done
    if (active) {
      // lane task p: channels 8 (p % 4) .. +7 at x = 2 (p / 4) and x + 1,
      // stored as BF16 pairs (x, x + 1) per channel
      const uint4* src = reinterpret_cast<const uint4*>(v + (size_t)row * nx * kC);
      for (int p = lane; p < 2 * nx; p += 64) {
        const int x = 2 * (p / 4), g = p % 4;
        const uint4 q0 = src[x * 4 + g], q1 = src[(x + 1) * 4 + g];
        const uint32_t w0[4] = {q0.x, q0.y, q0.z, q0.w}, w1[4] = {q1.x, q1.y, q1.z, q1.w};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const uint32_t lo = (w0[q / 2] >> (16 * (q % 2))) & 0xffffu;
          const uint32_t hi = (w1[q / 2] >> (16 * (q % 2))) & 0xffffu;
          tdw[(8 * g + q) * pdw + x / 2] = lo | (hi << 16);
        }
      }
    }
    __syncthreads();
    if (active) {
      f32x16 acc = {};
      for (int x0 = 0; x0 < nx; x0 += 16) {
        const bf16x8 b = load8(t + i * pitch + x0 + kb);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load8(wf + i * pitch + x0 + kb), b, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load8(wf + (32 + i) * pitch + x0 + kb), b, acc, 0, 0, 0);
      }
      float* out = a.X1 + (size_t)row * m2 * kC;
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) {
        const int j = mfma_row(rr, lane);
        if (j < m2) out[j * kC + i] = acc[rr];
      }
    }
  }
}

// ---------------------------------------------------- y and z sums
// Complex sums along an axis of a [..][n][m][2][C] array for one (outer, kx):
// forward: out[kk] = sum_t in[t] e^{-2 pi i k(kk) t / n} over the 2m kept k;
// inverse: out[t] = sum_kk in[kk] e^{+2 pi i k(kk) t / n}.
// One block per (outer, kx); the input column is staged in LDS. NT threads:
// groups of kC lanes take the outputs in turn (24 groups: one kept mode each
// at 2m = 24 forward; 32 groups for the inverse), so a block has enough
// waves to hide the LDS latency of its sums.
template <bool FWD> constexpr int ysum_threads() { return FWD ? 768 : 1024; }

template <bool FWD>
__global__ __launch_bounds__(ysum_threads<FWD>()) void k_ysum(const FArgs a, const float* __restrict__ in,
                                                              float* __restrict__ out) {
  constexpr int NT = ysum_threads<FWD>(), NG = NT / kC;
  extern __shared__ float sm[];
  const int ny = a.ny, m = a.m, my = 2 * m;
  const int nin = FWD ? ny : my, nout = FWD ? my : ny;
  float* col = sm;                                        // [nin][2][C]
  float2* tw = reinterpret_cast<float2*>(sm + nin * 2 * kC);  // [ny]
  const int z = blockIdx.x / m, kx = blockIdx.x % m;
  const size_t in_base = (size_t)z * nin * m * 2 * kC + (size_t)kx * 2 * kC;
  const size_t out_base = (size_t)z * nout * m * 2 * kC + (size_t)kx * 2 * kC;
  for (int i = threadIdx.x; i < nin * 2 * kC; i += NT) {
    const int t = i / (2 * kC), e = i % (2 * kC);
    col[i] = in[in_base + (size_t)t * m * 2 * kC + e];
  }
  for (int i = threadIdx.x; i < ny; i += NT) tw[i] = a.twy[i];
  __syncthreads();
  const int c = threadIdx.x % kC, g = threadIdx.x / kC;
  for (int o = g; o < nout; o += NG) {
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
      int j = 0;  // k(kk) o mod ny
      for (int kk = 0; kk < my; ++kk) {
        if (kk == m) j = inv_start(m, o, ny);
        const float2 w = tw[j];  // conjugate for the inverse
        const float xr = col[(2 * kk) * kC + c], xi = col[(2 * kk + 1) * kC + c];
        re += xr * w.x + xi * w.y;
        im += xi * w.x - xr * w.y;
        j += o;
        if (j >= ny) j -= ny;
      }
    }
    out[out_base + (size_t)o * m * 2 * kC + c] = re;
    out[out_base + (size_t)o * m * 2 * kC + kC + c] = im;
  }
}

// z pass: one block per kept (ky', kx): forward z sums to the 2m kept kz,
// channel mixing by R(kz', ky', kx) (complex, C x C, BF16), inverse z sums.
// There are only 2m^2 blocks (288 at m = 12), so each has kZmixThreads
// threads (32 groups of kC lanes) to keep the chip's SIMDs busy.
constexpr int kZmixThreads = 1024;

__global__ __launch_bounds__(kZmixThreads) void k_zmix(const FArgs a, const uint16_t* __restrict__ R) {
  constexpr int NT = kZmixThreads, NG = NT / kC;
  extern __shared__ float sm[];
  const int nz = a.nz, m = a.m, my = 2 * m;
  float* col = sm;                                // [nz][2][C]
  float* zs = col + nz * 2 * kC;                  // [2m][2][C]
  float* os = zs + my * 2 * kC;                   // [2m][2][C]
  float2* tw = reinterpret_cast<float2*>(os + my * 2 * kC);  // [nz]
  const int kyy = blockIdx.x / m, kx = blockIdx.x % m;
  const size_t zstride = (size_t)my * m * 2 * kC;
  const size_t base = (size_t)kyy * m * 2 * kC + (size_t)kx * 2 * kC;
  for (int i = threadIdx.x; i < nz * 2 * kC; i += NT) {
    const int t = i / (2 * kC), e = i % (2 * kC);
    col[i] = a.X2[base + (size_t)t * zstride + e];
  }
  for (int i = threadIdx.x; i < nz; i += NT) tw[i] = a.twz[i];
  __syncthreads();
  const int c = threadIdx.x % kC, g = threadIdx.x / kC;
  for (int kk = g; kk < my; kk += NG) {
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
  for (int kk = g; kk < my; kk += NG) {
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
  for (int t = g; t < nz; t += NG) {
    float re = 0.f, im = 0.f;
    int j = 0;  // k(kk) t mod nz
    for (int kk = 0; kk < my; ++kk) {
      if (kk == m) j = inv_start(m, t, nz);
      const float2 w = tw[j];
      const float xr = os[(2 * kk) * kC + c], xi = os[(2 * kk + 1) * kC + c];
      re += xr * w.x + xi * w.y;
      im += xi * w.x - xr * w.y;
      j += t;
      if (j >= nz) j -= nz;
    }
    a.Y2[base + (size_t)t * zstride + c] = re;
    a.Y2[base + (size_t)t * zstride + kC + c] = im;
  }
}

// ------------------------------------------- x inverse + local mixing
// v'[x][o] = GELU(sum_i W[o][i] v[x][i] + b[o] + sum_j WI[x][j] Y1[j][o]) with
// WI[x][2 kx] = s w cos(2 pi kx x / nx), WI[x][2 kx + 1] = -s w sin(2 pi kx x / nx),
// s = 1 / (nx ny nz), w = 1 (kx = 0) or 2, columns j >= 2m zero: the real
// part of the inverse x sum (the kx = 0 imaginary part drops out). The sum
// is a second product into the mixing's accumulator, with WI and Y1 (FP32)
// as BF16 hi and lo parts: A = WI (LDS), B = Y1 transposed to [o][j] in LDS.
// A block takes kInvRows rows per group; its waves share the 32-voxel tiles.
constexpr int kInvRows = 4, kInvGroups = 4;
constexpr int kYPitch = 40;  // bf16 per LDS row of the 32-wide j axis, a 16-byte multiple

__global__ __launch_bounds__(256) void k_xinv_mix(const FArgs a, const uint16_t* __restrict__ vin,
                                                  uint16_t* __restrict__ vout, const uint16_t* __restrict__ Wm,
                                                  const float* __restrict__ bias) {
  extern __shared__ __align__(16) uint16_t xs[];
  const int nx = a.nx;
  uint16_t* wi = xs;                         // [hi, lo][nx][kYPitch]
  uint16_t* yt = xs + 2 * nx * kYPitch;      // [kInvRows][hi, lo][32 o][kYPitch]
  for (int i = threadIdx.x; i < 2 * nx * 4; i += 256) {
    const int hx = i / 4, q = i % 4;  // hx = h * nx + x; four 16-byte pieces per x
    *reinterpret_cast<uint4*>(wi + hx * kYPitch + 8 * q) =
        *reinterpret_cast<const uint4*>(a.wxi + (size_t)hx * 32 + 8 * q);
  }
  const int rows = a.ny * a.nz, m2 = 2 * a.m, ntile = nx / 32;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int i = lane % 32, kb = 8 * (lane / 32);
  float bo[16];  // the bias of the output each accumulator holds
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) bo[rr] = bias[mfma_row(rr, lane)];
  for (int g = 0; g < kInvGroups; ++g) {
    const int row0 = (blockIdx.x * kInvGroups + g) * kInvRows;
    __syncthreads();  // the twiddles are in place; the previous group's reads are done
    for (int e = threadIdx.x; e < kInvRows * 32 * 32; e += 256) {
      const int rl = e / 1024, j = (e / 32) % 32, o = e % 32;
      const int row = row0 + rl;
      const float y = (row < rows && j < m2) ? a.Y1[((size_t)row * m2 + j) * kC + o] : 0.f;
      const uint16_t h = f2bf(y);
      yt[((rl * 2) * 32 + o) * kYPitch + j] = h;
      yt[((rl * 2 + 1) * 32 + o) * kYPitch + j] = f2bf(y - bf2f(h));
    }
    __syncthreads();
    for (int u = wave; u < kInvRows * ntile; u += 4) {
      const int rl = u / ntile, x0 = 32 * (u % ntile);
      const int row = row0 + rl;
      if (row >= rows) continue;  // uniform over the wave; no barrier follows in this loop
      const uint16_t* vrow = vin + (size_t)row * nx * kC;
      f32x16 acc = mix32(vrow, x0, Wm, lane);
      // the inverse x sum as the second product, transposed like the mixing:
      // A = Y1 [o][j] (hi, lo), B = WI^T [j][x] (hi, lo)
#pragma unroll
      for (int j0 = 0; j0 < 32; j0 += 16) {
        const bf16x8 wh = load8(wi + (x0 + i) * kYPitch + j0 + kb);
        const bf16x8 wl = load8(wi + (nx + x0 + i) * kYPitch + j0 + kb);
        const bf16x8 yh = load8(yt + ((rl * 2) * 32 + i) * kYPitch + j0 + kb);
        const bf16x8 yl = load8(yt + ((rl * 2 + 1) * 32 + i) * kYPitch + j0 + kb);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(yh, wh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(yl, wh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(yh, wl, acc, 0, 0, 0);
      }
      // lane: voxel x0 + i, outputs 8 g + 4 (lane / 32) .. +3 for g = 0..3: 8 bytes each
      uint16_t* ov = vout + ((size_t)row * nx + x0 + i) * kC + 4 * (lane / 32);
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        uint32_t w[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int rr = 4 * g + 2 * h;
          w[h] = (uint32_t)f2bf(gelu(acc[rr] + bo[rr])) | ((uint32_t)f2bf(gelu(acc[rr + 1] + bo[rr + 1])) << 16);
        }
        *reinterpret_cast<uint2*>(ov + 8 * g) = make_uint2(w[0], w[1]);
      }
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
  // accumulator rr of lane l: hidden unit h0 + mfma_row(rr, l) of voxel x0 + l % 32;
  // a lane sums its 16 units of each block of 32, its partner lane l ^ 32 the other 16
  float part = 0.f;
  const uint16_t* vt = v + x0 * kC;
  for (int h0 = 0; h0 < kH; h0 += 32) {
    const f32x16 acc = mix32(vt, 0, a.Q1 + (size_t)h0 * kC, lane);
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      const int h = h0 + mfma_row(rr, lane);
      part += a.Q2[h] * gelu(acc[rr] + a.q1[h]);
    }
  }
  part += __shfl_xor(part, 32, 64);
  if (lane < 32) {
    const size_t x = x0 + lane;
    out[x] = eta[x] + part + a.q2;
  }
}

}  // namespace pfn

// ====================================================================== host
namespace pfn {

size_t lds_xdft(const FArgs& a) { return (size_t)(2 + 4) * 32 * (a.nx + 8) * 2; }
size_t lds_ysum(const FArgs& a, bool fwd) {
  return (size_t)(fwd ? a.ny : 2 * a.m) * 2 * kC * 4 + (size_t)a.ny * 8;
}
size_t lds_zmix(const FArgs& a) { return ((size_t)a.nz + 4 * a.m) * 2 * kC * 4 + (size_t)a.nz * 8; }
size_t lds_xinv(const FArgs& a) { return ((size_t)2 * a.nx + kInvRows * 2 * 32) * kYPitch * 2; }

hipError_t forward(const FArgs& a, const float* eta_in, float* eta_out, hipStream_t s) {
  const int rows = a.nz * a.ny;
  k_lift<<<(unsigned)((a.nvox + 255) / 256), 256, 0, s>>>(a, eta_in, a.va);
  uint16_t* vin = a.va;
  uint16_t* vout = a.vb;
  for (int l = 0; l < kLayers; ++l) {
    k_xdft<<<(rows + 4 * kDftRounds - 1) / (4 * kDftRounds), 256, lds_xdft(a), s>>>(a, vin);
    k_ysum<true><<<a.nz * a.m, ysum_threads<true>(), lds_ysum(a, true), s>>>(a, a.X1, a.X2);
    k_zmix<<<2 * a.m * a.m, kZmixThreads, lds_zmix(a), s>>>(a, a.R + (size_t)l * a.r_stride);
    k_ysum<false><<<a.nz * a.m, ysum_threads<false>(), lds_ysum(a, false), s>>>(a, a.Y2, a.Y1);
    k_xinv_mix<<<(rows + kInvRows * kInvGroups - 1) / (kInvRows * kInvGroups), 256, lds_xinv(a), s>>>(
        a, vin, vout, a.W + (size_t)l * kC * kC, a.b + (size_t)l * kC);
    uint16_t* t = vin;
    vin = vout;
    vout = t;
  }
  k_proj<<<(unsigned)((a.nvox / 32 + 3) / 4), 256, 0, s>>>(a, vin, eta_in, eta_out);
  return hipGetLastError();
}

}  // namespace pfn
