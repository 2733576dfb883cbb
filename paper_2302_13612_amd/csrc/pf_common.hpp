// Device helpers shared by the x-pass kernels: block reductions, the
// per-voxel constitutive law, the real-to-complex split and merge of a row.
#pragma once
#include "fft_engine.hpp"
#include "pf_device.hpp"

namespace pft {

// -------------------------------------------------------------- reductions
template <int Q>
__device__ __forceinline__ void block_sum(double (&v)[Q], double* __restrict__ out) {
  __shared__ double red[16][Q];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < Q; ++q) red[wave][q] = v[q];
  __syncthreads();
  if (threadIdx.x < Q) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ void block_minmax(float mn, float mx, float* __restrict__ out) {
  __shared__ float red[16][2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mn = fminf(mn, __shfl_xor(mn, off, 64));
    mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  }
  if (lane == 0) {
    red[wave][0] = mn;
    red[wave][1] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = red[0][0], b = red[0][1];
    for (int w = 1; w < nw; ++w) {
      a = fminf(a, red[w][0]);
      b = fmaxf(b, red[w][1]);
    }
    out[0] = a;
    out[1] = b;
  }
  __syncthreads();
}

// -------------------------------------------------------------- material
// s = C g for a packed symmetric 6x6 C.
template <class TP>
__device__ __forceinline__ void symv6(TP C, const float g[6], float s[6]) {
  s[0] = C[0] * g[0] + C[1] * g[1] + C[2] * g[2] + C[3] * g[3] + C[4] * g[4] + C[5] * g[5];
  s[1] = C[1] * g[0] + C[6] * g[1] + C[7] * g[2] + C[8] * g[3] + C[9] * g[4] + C[10] * g[5];
  s[2] = C[2] * g[0] + C[7] * g[1] + C[11] * g[2] + C[12] * g[3] + C[13] * g[4] + C[14] * g[5];
  s[3] = C[3] * g[0] + C[8] * g[1] + C[12] * g[2] + C[15] * g[3] + C[16] * g[4] + C[17] * g[5];
  s[4] = C[4] * g[0] + C[9] * g[1] + C[13] * g[2] + C[16] * g[3] + C[18] * g[4] + C[19] * g[5];
  s[5] = C[5] * g[0] + C[10] * g[1] + C[14] * g[2] + C[17] * g[3] + C[19] * g[4] + C[20] * g[5];
}

__device__ __forceinline__ float h_of(float f, int kind) {
  return kind == 0 ? f : f * f * f * (6.f * f * f - 15.f * f + 10.f);
}
__device__ __forceinline__ float dh_of(float f, int kind) {
  return kind == 0 ? 1.f : 30.f * f * f * (f - 1.f) * (f - 1.f);
}

// Per-grain table: [C_g packed 21][dC_a packed 21 x V][eps0_a 6 x V].
template <int V>
struct Mat {
  float el[6];   // elastic strain (tensor-Voigt)
  float gam[6];  // elastic strain, engineering shear
  float sig[6];  // stress
};

// Elastic strain and stress of one voxel: eps* = eps_p + sum h(f_a) eps0_a,
// C(x) = C_g + sum h(f_a) dC_a, sigma = C(x) : (eps - eps*).
template <int V, class TP>
__device__ __forceinline__ void constitutive(const float e[6], const float eta[V], const float ep[6],
                                             TP tab, int h_kind, Mat<V>& o) {
  float h[V];
#pragma unroll
  for (int q = 0; q < V; ++q) h[q] = h_of(eta[q], h_kind);
  const TP e0 = tab + 21 * (V + 1);
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    float es = ep[c];
#pragma unroll
    for (int q = 0; q < V; ++q) es += h[q] * e0[6 * q + c];
    o.el[c] = e[c] - es;
    o.gam[c] = c < 3 ? o.el[c] : 2.f * o.el[c];
  }
  float Cx[21];
#pragma unroll
  for (int i = 0; i < 21; ++i) {
    float v = tab[i];
#pragma unroll
    for (int q = 0; q < V; ++q) v += h[q] * tab[21 * (q + 1) + i];
    Cx[i] = v;
  }
  symv6(Cx, o.gam, o.sig);
}

// ----------------------------------------------------------- x pass parts
// Forward: the NC complex rows held in v (packed real pairs) -> R2C spectra.
template <int M, int NC>
__device__ __forceinline__ void r2c_rows(float2 (&v)[NC][XPlan<M>::E], float2* ldsrow, int t, bool valid,
                                         float2* __restrict__ spec, size_t rowoff, size_t cstride,
                                         const float2* __restrict__ tw_m,
                                         const float2* __restrict__ tw_n) {
  constexpr int E = XPlan<M>::E, T = M / E;
  RowView view{ldsrow};
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    fft_pencil<M, 1, XPlan<M>>(v[c], view, t, tw_m);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) view.write(t + T * m, v[c][m]);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int k = t + T * m;
      const float2 zk = v[c][m];
      const float2 zm = view.read(k == 0 ? 0 : M - k);
      // X[k] = E[k] + W_N^k O[k]; E = (Z_k + conj Z_{M-k})/2, O = -i (Z_k - conj Z_{M-k})/2
      const float2 ev = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
      const float2 d = make_float2(zk.x - zm.x, zk.y + zm.y);
      const float2 od = make_float2(0.5f * d.y, -0.5f * d.x);
      const float2 X = cadd(ev, cmul(tw_n[k], od));
      if (valid) spec[c * cstride + rowoff + k] = X;
    }
    if (t == 0 && valid) spec[c * cstride + rowoff + M] = make_float2(v[c][0].x - v[c][0].y, 0.f);
  }
}

// Inverse: one spectral row (M+1 coefficients) -> packed real pairs in v
// (unnormalised); the imaginary parts of the kx = 0 and kx = M terms are
// ignored, as for the spectrum of a real field.
template <int M>
__device__ __forceinline__ void c2r_row(float2 (&v)[XPlan<M>::E], float2* ldsrow, int t, bool valid,
                                        const float2* __restrict__ srow,
                                        const float2* __restrict__ tw_m,
                                        const float2* __restrict__ tw_n) {
  constexpr int E = XPlan<M>::E, T = M / E;
  RowView view{ldsrow};
  __syncthreads();
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = t + T * m;
    view.write(k, valid ? srow[k] : make_float2(0.f, 0.f));
  }
  if (t == 0) view.write(M, valid ? srow[M] : make_float2(0.f, 0.f));
  __syncthreads();
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = t + T * m;
    float2 X = view.read(k);
    float2 Xm = view.read(M - k);
    if (k == 0) {
      X.y = 0.f;
      Xm.y = 0.f;
    }
    // Z = (X_k + conj X_{M-k}) + i W_N^{-k} (X_k - conj X_{M-k})
    const float2 ev = make_float2(X.x + Xm.x, X.y - Xm.y);
    const float2 od = cmul(make_float2(X.x - Xm.x, X.y + Xm.y), cconj(tw_n[k]));
    v[m] = make_float2(ev.x - od.y, ev.y + od.x);
  }
  fft_pencil<M, -1, XPlan<M>>(v, view, t, tw_m);
}

// Per-voxel material table of grain g. When the whole wavefront sits in one
// grain the table is read through the constant address space (scalar loads
// into SGPRs); otherwise through per-lane global loads.
typedef const __attribute__((address_space(4))) float* ctab_t;
typedef const __attribute__((address_space(1))) float* gtab_t;

template <class F>
__device__ __forceinline__ void with_table(const KArgs& a, int g, F&& f) {
  const int gu = __builtin_amdgcn_readfirstlane(g);
  if (__all(g == gu)) {
    f((ctab_t)(a.tables + gu * a.tab_stride));
  } else {
    f((gtab_t)(a.tables + g * a.tab_stride));
  }
}

}  // namespace pft
