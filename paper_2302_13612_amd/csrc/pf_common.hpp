// Device helpers shared by the x-pass kernels: block reductions, the
// per-voxel constitutive law, the real-to-complex split and merge of a row.
#pragma once
#include "fft_engine.hpp"
#include "pf_device.hpp"

namespace pft {

// Pointer into read-only memory that is the same for every lane (constant
// address space): loads through it with a uniform address are scalar loads.
typedef const __attribute__((address_space(4))) float* ctab_t;

// -------------------------------------------------------------- reductions
// NW: the most wavefronts a calling block has (its LDS scratch is sized by
// it; the x passes' staging leaves little LDS to spare at three blocks/CU).
template <int Q, int NW = 16>
__device__ __forceinline__ void block_sum(double (&v)[Q], double* __restrict__ out) {
  __shared__ double red[NW][Q];
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

template <int NW = 16>
__device__ __forceinline__ void block_minmax(float mn, float mx, float* __restrict__ out) {
  __shared__ float red[NW][2];
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

// Reciprocal by the hardware instruction (within 1 ulp): the spectral
// passes divide by a per-wavevector determinant or denominator at every
// element, where a correctly rounded division costs about ten instructions.
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

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

// Rotation form of the constitutive law for a polycrystal whose grains share
// one crystal-frame material: the elastic strain is turned into the crystal
// frame of the voxel's grain (e_c = R^T e R), the crystal-frame mixture
// stiffness and twin eigenstrains (wave-uniform constants) give the stress,
// which is turned back (sigma = R sigma_c R^T).
template <int V>
struct MatR {
  float gam_c[6];  // elastic strain in the crystal frame, engineering shear
  float sig_c[6];  // stress in the crystal frame
  float sig[6];    // stress in the sample frame
};

// out = R^T A R (to_crystal) or R A R^T, A symmetric (tensor-Voigt).
template <bool TO_CRYSTAL>
__device__ __forceinline__ void rotate_sym(const float (&R)[9], const float (&A)[6], float (&out)[6]) {
  const float M[3][3] = {{A[0], A[5], A[4]}, {A[5], A[1], A[3]}, {A[4], A[3], A[2]}};
  float B[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < 3; ++k) acc += M[i][k] * (TO_CRYSTAL ? R[3 * k + j] : R[3 * j + k]);
      B[i][j] = acc;
    }
  constexpr int PI[6] = {0, 1, 2, 1, 0, 0}, PJ[6] = {0, 1, 2, 2, 2, 1};
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const int i = PI[c], j = PJ[c];
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) acc += (TO_CRYSTAL ? R[3 * k + i] : R[3 * i + k]) * B[k][j];
    out[c] = acc;
  }
}

// The crystal-frame table of the rotation form, read with scalar loads from
// kernel-argument memory: each
// element goes through the constant cache into a scalar register and costs
// no vector instruction. The table does not fit in scalar registers, so it
// is read block by block where it is used, and each block's base pointer
// passes through an opaque scalar zero that waits for a value of the block
// before: the loads cannot be hoisted out of the voxel loop or bunched at
// its top (either would spill the table to vector lanes), and one block's
// loads overlap the arithmetic of the one before.
__device__ __forceinline__ ctab_t smem_after(ctab_t p, float dep) {
  int zero;
  asm volatile("s_mov_b32 %0, 0" : "=s"(zero) : "v"(dep));
  return p + zero;
}

// The crystal table inside the kernel's argument block, for kernels whose
// only explicit argument is the KArgs block (which then sits at offset 0 of
// the argument segment). Addressing it this way leaves the by-value
// parameter's address untaken: a taken address can make the compiler copy
// the whole block to scratch memory.
__device__ __forceinline__ ctab_t kernarg_xtab() {
  typedef const __attribute__((address_space(4))) char* cbyte_t;
  return (ctab_t)((cbyte_t)__builtin_amdgcn_kernarg_segment_ptr() + offsetof(KArgs, xtab));
}

// Rotation-form constitutive law of the two voxels of a packed sample, the
// crystal table read with scalar loads (layout as for constitutive_rot).
template <int V>
__device__ __forceinline__ void constitutive_rot_pair(ctab_t xtab, int hk, const float (&e)[2][6],
                                                      const float (&eta)[2][V], const float (&ep)[2][6],
                                                      const float (&R)[2][9], MatR<V> (&o)[2]) {
  float h[2][V], dc[2][6];
#pragma unroll
  for (int v = 0; v < 2; ++v) {
#pragma unroll
    for (int q = 0; q < V; ++q) h[v][q] = h_of(eta[v][q], hk);
    float d[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) d[c] = e[v][c] - ep[v][c];
    rotate_sym<true>(R[v], d, dc[v]);
  }
  ctab_t t = smem_after(xtab + 21 * (V + 1), dc[1][0]);
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      float es = 0.f;
#pragma unroll
      for (int q = 0; q < V; ++q) es += h[v][q] * t[6 * q + c];
      const float el = dc[v][c] - es;
      o[v].gam_c[c] = c < 3 ? el : 2.f * el;
    }
  float Cx[2][21];
  t = smem_after(xtab, o[1].gam_c[0]);
#pragma unroll
  for (int i = 0; i < 21; ++i) Cx[0][i] = Cx[1][i] = t[i];
#pragma unroll
  for (int q = 0; q < V; ++q) {
    t = smem_after(xtab + 21 * (q + 1), Cx[1][10]);
#pragma unroll
    for (int i = 0; i < 21; ++i)
#pragma unroll
      for (int v = 0; v < 2; ++v) Cx[v][i] += h[v][q] * t[i];
  }
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    symv6(Cx[v], o[v].gam_c, o[v].sig_c);
    rotate_sym<false>(R[v], o[v].sig_c, o[v].sig);
  }
}

__device__ __forceinline__ void load_rotation(const KArgs& a, int g, float (&R)[9]) {
  const float4* r = reinterpret_cast<const float4*>(a.rot + 12 * g);
  const float4 r0 = r[0], r1 = r[1], r2 = r[2];
  R[0] = r0.x; R[1] = r0.y; R[2] = r0.z; R[3] = r0.w;
  R[4] = r1.x; R[5] = r1.y; R[6] = r1.z; R[7] = r1.w;
  R[8] = r2.x;
}

// ----------------------------------------------------------- x pass parts
// Rows of the x passes are exchanged with wavefront order only (RowView).
template <int M>
constexpr bool row_in_wave() { return 64 % (M / XPlan<M>::E) == 0; }

// Threads per x-pass block for half-length M (smaller for the radix-3 rows so
// the staging slabs stay within 64 KiB of LDS).
template <int M>
__host__ __device__ constexpr int xthreads() { return (M % 3 == 0) ? 128 : 256; }

// Forward: the NC complex rows held in v (packed real pairs) -> R2C spectra.
template <int M, int NC>
__device__ __forceinline__ void r2c_rows(float2 (&v)[NC][XPlan<M>::E], float2* ldsrow, int t, bool valid,
                                         float2* __restrict__ spec, size_t rowoff, size_t cstride,
                                         float2* __restrict__ nq, const float2* __restrict__ tw_m,
                                         const float2* __restrict__ tw_n) {
  constexpr int E = XPlan<M>::E, T = M / E;
  static_assert(row_in_wave<M>(), "the threads of a row must lie in one wavefront");
  RowView view{ldsrow};
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    fft_pencil<M, 1, XPlan<M>>(v[c], view, t, tw_m);
    view.sync();
#pragma unroll
    for (int m = 0; m < E; ++m) view.write(t + T * m, v[c][m]);
    view.sync();
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
      if (valid) gst(spec + c * cstride + rowoff + k, X);
    }
    if (t == 0 && valid) gst(nq + c * cstride, make_float2(v[c][0].x - v[c][0].y, 0.f));
  }
}

// Twiddles a thread uses on every row of an x pass: those of the
// half-length FFT in direction DIR and the split factors W_N^k of its own
// k = t + T m (taken as stored; the inverse conjugates them where used).
// Loaded once per kernel, they keep the row transforms free of table loads.
template <int M, int DIR>
struct XTw {
  static_assert(row_in_wave<M>(), "the threads of a row must lie in one wavefront");
  TwCache<M, XPlan<M>, DIR> fft;
  float2 split[XPlan<M>::E];
  __device__ __forceinline__ void load(const KArgs& a, int t) {
    constexpr int E = XPlan<M>::E, T = M / E;
    fft.load(a.tw_xh, t);
#pragma unroll
    for (int m = 0; m < E; ++m) split[m] = a.tw_x[t + T * m];
  }
};

// Forward of one staged row: v (packed real pairs) -> FFT -> split into the
// nx/2+1 coefficients, kx < nx/2 stored at dst, kx = nx/2 at nq. ldsrow is
// this row's exchange buffer.
template <int M>
__device__ __forceinline__ void r2c_one(float2 (&v)[XPlan<M>::E], float2* ldsrow, int t, bool valid,
                                        float2* __restrict__ dst, float2* __restrict__ nq, const XTw<M, 1>& tw) {
  constexpr int E = XPlan<M>::E, T = M / E;
  RowView view{ldsrow};
  fft_pencil<M, 1, XPlan<M>>(v, view, t, tw.fft);
  view.sync();
#pragma unroll
  for (int m = 0; m < E; ++m) view.write(t + T * m, v[m]);
  view.sync();
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = t + T * m;
    const float2 zk = v[m];
    const float2 zm = view.read(k == 0 ? 0 : M - k);
    const float2 ev = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
    const float2 d = make_float2(zk.x - zm.x, zk.y + zm.y);
    const float2 od = make_float2(0.5f * d.y, -0.5f * d.x);
    const float2 X = cadd(ev, cmul(tw.split[m], od));
    if (valid) gst(dst + k, X);
  }
  if (t == 0 && valid) gst(nq, make_float2(v[0].x - v[0].y, 0.f));
}

// Inverse of one spectral row, in two parts so the global loads of the next
// row can be issued before the current one is transformed:
// c2r_fetch loads the M+1 coefficients a thread needs into registers;
// c2r_from_regs builds the packed half-length spectrum through LDS and runs
// the inverse FFT (unnormalised). The imaginary parts of the kx = 0 and
// kx = M terms are ignored, as for the spectrum of a real field.
template <int M>
struct RowFetch {
  float2 x[XPlan<M>::E];
  float2 last;  // coefficient M (thread 0 only)
};

template <int M>
__device__ __forceinline__ void c2r_fetch(RowFetch<M>& f, int t, bool valid, const float2* __restrict__ srow,
                                          const float2* __restrict__ nq) {
  constexpr int E = XPlan<M>::E, T = M / E;
#pragma unroll
  for (int m = 0; m < E; ++m) f.x[m] = valid ? gld(srow + t + T * m) : make_float2(0.f, 0.f);
  f.last = (valid && t == 0) ? gld(nq) : make_float2(0.f, 0.f);
}

template <int M>
__device__ __forceinline__ void c2r_from_regs(float2 (&v)[XPlan<M>::E], const RowFetch<M>& f, float2* ldsrow,
                                              int t, const XTw<M, -1>& tw) {
  constexpr int E = XPlan<M>::E, T = M / E;
  RowView view{ldsrow};
  view.sync();
#pragma unroll
  for (int m = 0; m < E; ++m) view.write(t + T * m, f.x[m]);
  if (t == 0) view.write(M, f.last);
  view.sync();
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
    const float2 od = cmul(make_float2(X.x - Xm.x, X.y + Xm.y), cconj(tw.split[m]));
    v[m] = make_float2(ev.x - od.y, ev.y + od.x);
  }
  fft_pencil<M, -1, XPlan<M>>(v, view, t, tw.fft);
}

template <int M>
__device__ __forceinline__ void c2r_row(float2 (&v)[XPlan<M>::E], float2* ldsrow, int t, bool valid,
                                        const float2* __restrict__ srow, const float2* __restrict__ nq,
                                        const XTw<M, -1>& tw) {
  RowFetch<M> f;
  c2r_fetch<M>(f, t, valid, srow, nq);
  c2r_from_regs<M>(v, f, ldsrow, t, tw);
}

// Per-voxel material table of grain g, always read through the constant
// address space with a wave-uniform address (scalar loads into SGPRs): the
// distinct grains of a wavefront are visited one after the other, each with
// only its lanes active (usually one grain, two or three at boundaries).

template <class F>
__device__ __forceinline__ void with_table(const KArgs& a, const float* base, int g, F&& f) {
  bool todo = true;
  while (true) {
    if (todo) {
      const int gu = __builtin_amdgcn_readfirstlane(g);
      if (g == gu) {
        f((ctab_t)(base + gu * a.tab_stride));
        todo = false;
      }
    }
    if (!__any(todo)) break;
  }
}

}  // namespace pft
