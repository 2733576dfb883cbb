// Spectral convolution of the Fourier neural operator for training (FP32,
// channel-first batches as the training model holds them):
//   forward   y = irfftn(embed(R . sub(rfftn(v))))            (K v)
//   backward  G  = c(kx)/N sub(rfftn(dy)),  dR = sum_b G conj(S),
//             dv = sum over kept modes Re[(R^H G) e^{+i theta}]
// with sub() the kept modes (kx < m; ky, kz in [0, m) u [n - m, n), positive
// then negative), c(kx) = 1 on the kx = 0 plane and 2 elsewhere, S the kept
// modes of v from the forward pass, dR holding dL/dRe R + i dL/dIm R. Only
// 2m x 2m x m modes are kept, so every transform is a truncated discrete
// Fourier sum along one axis (x: real rows to m modes; y, z: complex, to or
// from the 2m kept indices), each output one thread's sum over the axis.
//
// Layouts: v, y, dy, dv [B][C][nz][ny][nx] float; S, G [B][C][2m][2m][m]
// complex (re, im interleaved); R, dR [C][C][2m][2m][m] complex, indexed
// [out][in][kz'][ky'][kx].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pf.h"

namespace pfs {

constexpr int kMaxN = 256;

__device__ __forceinline__ int kept_freq(int kk, int m, int n) { return kk < m ? kk : n - 2 * m + kk; }

// e^{sign 2 pi i idx / n} from an exact table of n roots. A sum over one
// axis steps idx = (k j) mod n by k (or j), each step below n, with one
// wrap; an inverse sum over the kept list restarts at the negative
// frequencies from (n - m) j mod n = (-m j) mod n.
__device__ __forceinline__ float2 root(const float2* tw, int idx, int sign) {
  const float2 w = tw[idx];
  return make_float2(w.x, sign > 0 ? w.y : -w.y);
}

__device__ __forceinline__ int step_idx(int idx, int d, int n) {
  idx += d;
  return idx >= n ? idx - n : idx;
}

__device__ __forceinline__ int neg_start(int m, int j, int n) {
  const int r = (m * j) % n;
  return r == 0 ? 0 : n - r;
}

__device__ __forceinline__ void load_roots(float2* tw, int n) {
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    float s, c;
    sincospif(2.f * (float)j / (float)n, &s, &c);
    tw[j] = make_float2(c, s);
  }
  __syncthreads();
}

// x: X[r][kx] = scale c_kx sum_x v[r][x] e^{-2 pi i kx x / nx}, kx < m;
// c_kx = 1 unless weight_c and kx > 0 (then 2). 16 rows per block.
__global__ __launch_bounds__(256) void k_tx_fwd(const float* __restrict__ v, float2* __restrict__ X, long rows,
                                                int nx, int m, float scale, int weight_c) {
  __shared__ float2 tw[kMaxN];
  __shared__ float row[16][kMaxN];
  load_roots(tw, nx);
  const long r0 = (long)blockIdx.x * 16;
  for (int i = threadIdx.x; i < 16 * nx; i += blockDim.x) {
    const int rr = i / nx, x = i % nx;
    row[rr][x] = r0 + rr < rows ? v[(r0 + rr) * nx + x] : 0.f;
  }
  __syncthreads();
  for (int o = threadIdx.x; o < 16 * m; o += blockDim.x) {
    const int rr = o / m, kx = o % m;
    if (r0 + rr >= rows) continue;
    float re = 0.f, im = 0.f;
    int idx = 0;  // kx x mod nx
    for (int x = 0; x < nx; ++x) {
      const float2 w = root(tw, idx, -1);
      re += row[rr][x] * w.x;
      im += row[rr][x] * w.y;
      idx = step_idx(idx, kx, nx);
    }
    const float s = scale * ((weight_c && kx > 0) ? 2.f : 1.f);
    X[(r0 + rr) * m + kx] = make_float2(s * re, s * im);
  }
}

// along an axis of length n with stride inner: to the 2m kept indices
// (dir -1) or from them back to all n (dir +1):
//   dir -1: out[o][kk][i] = sum_j in[o][j][i] e^{-2 pi i f(kk) j / n}
//   dir +1: out[o][j][i]  = sum_kk in[o][kk][i] e^{+2 pi i f(kk) j / n}
__global__ __launch_bounds__(256) void k_t_axis(const float2* __restrict__ in, float2* __restrict__ out,
                                                long outer, int n, long inner, int m, int dir) {
  __shared__ float2 tw[kMaxN];
  load_roots(tw, n);
  const int nout = dir < 0 ? 2 * m : n, nin = dir < 0 ? n : 2 * m;
  const long total = outer * nout * inner;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const long i = t % inner;
    const int q = (int)((t / inner) % nout);
    const long o = t / (inner * nout);
    const float2* src = in + o * nin * inner + i;
    float re = 0.f, im = 0.f;
    // forward: q a kept index, p a grid index, idx = f(q) p mod n;
    // inverse: p a kept index, q a grid index, idx = f(p) q mod n
    const int d = dir < 0 ? kept_freq(q, m, n) : q;
    int idx = 0;
    for (int p = 0; p < nin; ++p) {
      if (dir > 0 && p == m) idx = neg_start(m, q, n);
      const float2 w = root(tw, idx, dir);
      const float2 a = src[(long)p * inner];
      re += a.x * w.x - a.y * w.y;
      im += a.x * w.y + a.y * w.x;
      idx = step_idx(idx, d, n);
    }
    out[t] = make_float2(re, im);
  }
}

// per kept mode k and batch item: out[b][o][k] = sum_i R[o][i][k] in[b][i][k],
// or with adjoint R^H: out[b][i][k] = sum_o conj(R[o][i][k]) in[b][o][k]
__global__ __launch_bounds__(256) void k_mix(const float2* __restrict__ R, const float2* __restrict__ in,
                                             float2* __restrict__ out, int B, int C, long K, int adjoint) {
  const long total = (long)B * C * K;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const long k = t % K;
    const int c = (int)((t / K) % C);
    const int b = (int)(t / (K * C));
    float re = 0.f, im = 0.f;
    for (int j = 0; j < C; ++j) {
      float2 r = adjoint ? R[((long)j * C + c) * K + k] : R[((long)c * C + j) * K + k];
      if (adjoint) r.y = -r.y;
      const float2 a = in[((long)b * C + j) * K + k];
      re += r.x * a.x - r.y * a.y;
      im += r.x * a.y + r.y * a.x;
    }
    out[t] = make_float2(re, im);
  }
}

// x back to real rows: y[r][x] = scale sum_{kx<m} c_kx Re[Y[r][kx] e^{+2 pi i kx x / nx}]
__global__ __launch_bounds__(256) void k_tx_inv(const float2* __restrict__ Y, float* __restrict__ y, long rows,
                                                int nx, int m, float scale, int weight_c) {
  __shared__ float2 tw[kMaxN];
  load_roots(tw, nx);
  const long total = rows * nx;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const long r = t / nx;
    const int x = (int)(t % nx);
    float acc = 0.f;
    int idx = 0;  // kx x mod nx
    for (int kx = 0; kx < m; ++kx) {
      const float2 a = Y[r * m + kx];
      const float2 w = root(tw, idx, +1);
      acc += ((weight_c && kx > 0) ? 2.f : 1.f) * (a.x * w.x - a.y * w.y);
      idx = step_idx(idx, x, nx);
    }
    y[t] = scale * acc;
  }
}

// dR[o][i][k] = sum_b G[b][o][k] conj(S[b][i][k])
__global__ __launch_bounds__(256) void k_outer(const float2* __restrict__ G, const float2* __restrict__ S,
                                               float2* __restrict__ dR, int B, int C, long K) {
  const long total = (long)C * C * K;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const long k = t % K;
    const int i = (int)((t / K) % C);
    const int o = (int)(t / (K * C));
    float re = 0.f, im = 0.f;
    for (int b = 0; b < B; ++b) {
      const float2 g = G[((long)b * C + o) * K + k];
      const float2 s = S[((long)b * C + i) * K + k];
      re += g.x * s.x + g.y * s.y;
      im += g.y * s.x - g.x * s.y;
    }
    dR[t] = make_float2(re, im);
  }
}

struct Dims {
  int B, C, nx, ny, nz, m;
  long rows_x() const { return (long)B * C * nz * ny; }
  long K() const { return 4L * m * m * m; }
  // work: X1 [B C nz][ny][m], X2 [B C nz][2m][m] (complex)
  size_t x1() const { return (size_t)B * C * nz * ny * m; }
  size_t x2() const { return (size_t)B * C * nz * 2 * m * m; }
};

int grid_for(long total) {
  const long b = (total + 255) / 256;
  return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

// v (real) -> kept modes S: x, then y, then z
hipError_t truncated_forward(const Dims& d, const float* v, float2* S, float2* X1, float2* X2, float scale,
                             int weight_c, hipStream_t s) {
  const long rows = d.rows_x();
  k_tx_fwd<<<(int)((rows + 15) / 16), 256, 0, s>>>(v, X1, rows, d.nx, d.m, scale, weight_c);
  k_t_axis<<<grid_for((long)d.B * d.C * d.nz * 2 * d.m * d.m), 256, 0, s>>>(
      X1, X2, (long)d.B * d.C * d.nz, d.ny, d.m, d.m, -1);
  k_t_axis<<<grid_for((long)d.B * d.C * d.K()), 256, 0, s>>>(X2, S, (long)d.B * d.C, d.nz, 2L * d.m * d.m, d.m,
                                                               -1);
  return hipGetLastError();
}

// kept modes O -> real y: z, then y, then x
hipError_t truncated_inverse(const Dims& d, const float2* O, float* y, float2* X1, float2* X2, float scale,
                             int weight_c, hipStream_t s) {
  k_t_axis<<<grid_for((long)d.B * d.C * d.nz * 2 * d.m * d.m), 256, 0, s>>>(O, X2, (long)d.B * d.C, d.nz,
                                                                              2L * d.m * d.m, d.m, +1);
  k_t_axis<<<grid_for((long)d.B * d.C * d.nz * d.ny * d.m), 256, 0, s>>>(X2, X1, (long)d.B * d.C * d.nz, d.ny,
                                                                          d.m, d.m, +1);
  const long rows = d.rows_x();
  k_tx_inv<<<grid_for(rows * d.nx), 256, 0, s>>>(X1, y, rows, d.nx, d.m, scale, weight_c);
  return hipGetLastError();
}

bool dims_ok(const Dims& d) {
  auto axis = [](int n) { return n >= 4 && n <= kMaxN; };
  return d.B >= 1 && d.B <= 64 && d.C >= 1 && d.C <= 256 && axis(d.nx) && axis(d.ny) && axis(d.nz) && d.m >= 1 &&
         2 * d.m < d.nx && 2 * d.m <= d.ny && 2 * d.m <= d.nz;
}

}  // namespace pfs

extern "C" {

int pf_specconv_workspace_size(int32_t B, int32_t C, int32_t nx, int32_t ny, int32_t nz, int32_t m,
                               size_t* bytes) {
  const pfs::Dims d{B, C, nx, ny, nz, m};
  if (!bytes || !pfs::dims_ok(d)) return PF_EINVAL;
  *bytes = sizeof(float2) * (d.x1() + d.x2() + 256);
  return PF_OK;
}

int pf_specconv_forward(int32_t B, int32_t C, int32_t nx, int32_t ny, int32_t nz, int32_t m, const float* v,
                        const float* R, float* S, float* M, float* y, void* work, size_t work_bytes,
                        void* hip_stream) {
  const pfs::Dims d{B, C, nx, ny, nz, m};
  if (!pfs::dims_ok(d) || !v || !R || !S || !M || !y || !work) return PF_EINVAL;
  if (work_bytes < sizeof(float2) * (d.x1() + d.x2())) return PF_ENOMEM;
  hipStream_t s = (hipStream_t)hip_stream;
  float2* X1 = (float2*)work;
  float2* X2 = X1 + d.x1();
  hipError_t e = pfs::truncated_forward(d, v, (float2*)S, X1, X2, 1.f, 0, s);
  if (e == hipSuccess) {
    const long total = (long)B * C * d.K();
    pfs::k_mix<<<pfs::grid_for(total), 256, 0, s>>>((const float2*)R, (const float2*)S, (float2*)M, B, C, d.K(), 0);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = pfs::truncated_inverse(d, (const float2*)M, y, X1, X2, 1.f / ((float)nx * ny * nz), 1, s);
  return e == hipSuccess ? PF_OK : PF_EDEVICE;
}

int pf_specconv_backward(int32_t B, int32_t C, int32_t nx, int32_t ny, int32_t nz, int32_t m, const float* dy,
                         const float* R, const float* S, float* G, float* M, float* dv, float* dR, void* work,
                         size_t work_bytes, void* hip_stream) {
  const pfs::Dims d{B, C, nx, ny, nz, m};
  if (!pfs::dims_ok(d) || !dy || !R || !S || !G || !M || !dv || !dR || !work) return PF_EINVAL;
  if (work_bytes < sizeof(float2) * (d.x1() + d.x2())) return PF_ENOMEM;
  hipStream_t s = (hipStream_t)hip_stream;
  float2* X1 = (float2*)work;
  float2* X2 = X1 + d.x1();
  // G = c(kx)/N times the kept modes of dy
  hipError_t e = pfs::truncated_forward(d, dy, (float2*)G, X1, X2, 1.f / ((float)nx * ny * nz), 1, s);
  if (e == hipSuccess) {
    const long cck = (long)C * C * d.K();
    pfs::k_outer<<<pfs::grid_for(cck), 256, 0, s>>>((const float2*)G, (const float2*)S, (float2*)dR, B, C, d.K());
    const long total = (long)B * C * d.K();
    pfs::k_mix<<<pfs::grid_for(total), 256, 0, s>>>((const float2*)R, (const float2*)G, (float2*)M, B, C, d.K(), 1);
    e = hipGetLastError();
  }
  // dv = sum over kept modes Re[(R^H G) e^{+i theta}]: the inverse sums without c or 1/N
  if (e == hipSuccess) e = pfs::truncated_inverse(d, (const float2*)M, dv, X1, X2, 1.f, 0, s);
  return e == hipSuccess ? PF_OK : PF_EDEVICE;
}

}  // extern "C"
