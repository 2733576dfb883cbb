// Forward x-pass kernels with the per-voxel physics, for PF_NV twin variants
// per voxel (this file is compiled once per PF_NV = 1..6).
//
// Two phases per block of rows:
//   1. every thread evaluates the physics of its voxels (two per packed
//      complex sample) and stages the outputs in LDS, one slab per output
//      component, at the positions its own FFT lanes read back;
//   2. for each component the row FFT runs from its slab, which then serves
//      as that transform's exchange buffer, and the split coefficients go to
//      HBM.
// The FFT data never share registers with the physics, which keeps register
// use low enough for three blocks per CU.
//
// Material: either per-grain sample-frame tables (any material), or, for a
// polycrystal of one crystal (ROT), the grain rotation per voxel and one
// crystal-frame table held in kernel arguments (scalar registers).
#include "pf_common.hpp"

#ifndef PF_NV
#error "PF_NV (number of twin variants) must be defined"
#endif
// waves per SIMD the forward x passes are compiled for (their LDS staging
// allows three blocks of 256 threads per CU)
constexpr int kXWaves = 3;

namespace pft {

// A scalar zero the compiler cannot see through: added to the component
// stride inside the voxel loop, it keeps the per-component base addresses
// from being hoisted out of the loop (held across it, they would not fit in
// scalar registers).
__device__ __forceinline__ int opaque_zero() {
  int zero;
  asm volatile("s_mov_b32 %0, 0" : "=s"(zero));
  return zero;
}

// A float2 of a field at a 32-bit element offset from a wave-uniform base:
// the load takes the base in scalar registers and only the offset in a
// vector register, so no 64-bit per-lane addresses are kept live. A field
// component holds fewer than 2^30 elements (the host checks the batch size).
__device__ __forceinline__ float2 ld_f2(const float* base, uint32_t elem) {
  return gld(reinterpret_cast<const float2*>(reinterpret_cast<const char*>(base) + (elem << 2)));
}

// Inputs of one packed sample (voxels x0, x0+1) of a row.
template <int V>
struct Sample {
  float2 e[6], p[6], h[V];
  int g0, g1;
};

template <int E> struct GidPack;

// Strain of the first iterate of a step: the stored (latest converged)
// field L, or its extrapolation from the converged fields of the previous
// steps: linear 2 L - P, quadratic 3 (L - P) + P2, cubic 4 (L + P2) - 6 P - P3.
// Rows past the end read row 0 (their results are not stored), so the
// loads need no per-lane condition.
__device__ __forceinline__ void extrapolate_strain(const KArgs& a, size_t vs, uint32_t off, float2 (&e)[6]) {
  if (a.iter_mode == 0) return;
  vs += opaque_zero();
  // every load of a mode is issued before its arithmetic (the mode is
  // uniform, the branches do not wait on memory)
  float2 p1[6], p2[6], p3[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) p1[c] = ld_f2(a.eps_h1 + c * vs, off);
  if (a.iter_mode == 1) {
#pragma unroll
    for (int c = 0; c < 6; ++c) e[c] = make_float2(2.f * e[c].x - p1[c].x, 2.f * e[c].y - p1[c].y);
    return;
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) p2[c] = ld_f2(a.eps_h2 + c * vs, off);
  if (a.iter_mode == 2) {
#pragma unroll
    for (int c = 0; c < 6; ++c)
      e[c] = make_float2(3.f * (e[c].x - p1[c].x) + p2[c].x, 3.f * (e[c].y - p1[c].y) + p2[c].y);
    return;
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) p3[c] = ld_f2(a.eps_h3 + c * vs, off);
#pragma unroll
  for (int c = 0; c < 6; ++c)
    e[c] = make_float2(4.f * (e[c].x + p2[c].x) - 6.f * p1[c].x - p3[c].x,
                       4.f * (e[c].y + p2[c].y) - 6.f * p1[c].y - p3[c].y);
}

// Offset added to the strain the iterate is formed from so its mean is the
// iterate's prescribed mean.
__device__ __forceinline__ float mean_shift(const KArgs& a, const DevState* st, int c) {
  return (float)(st->ebar_cur[c] - st->ebar_base[c]);
}

template <int V>
__device__ __forceinline__ void load_sample(const KArgs& a, size_t vs, uint32_t off, Sample<V>& s) {
  s.g0 = s.g1 = 0;
  vs += opaque_zero();
#pragma unroll
  for (int c = 0; c < 6; ++c) s.e[c] = ld_f2(a.eps + c * vs, off);
#pragma unroll
  for (int q = 0; q < V; ++q) s.h[q] = ld_f2(a.eta + q * vs, off);
  if (a.epsp) {
#pragma unroll
    for (int c = 0; c < 6; ++c) s.p[c] = ld_f2(a.epsp + c * vs, off);
  } else {
#pragma unroll
    for (int c = 0; c < 6; ++c) s.p[c] = make_float2(0.f, 0.f);
  }
}

// Grain ids of a thread's E samples (one byte per voxel, two per sample),
// loaded before the voxel loop so that each iteration's rotation gathers
// leave together with its field loads instead of waiting for the id load.
template <int E>
struct GidPack {
  uint64_t lo = 0;  // samples 0..3
  uint32_t hi = 0;  // samples 4, 5
  __device__ __forceinline__ void load(const KArgs& a, size_t rbase, int t, int T) {
    if (!a.gid) return;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const uint32_t gg = *reinterpret_cast<const uint16_t*>(a.gid + rbase + 2 * (t + T * m));
      if (m < 4) lo |= (uint64_t)gg << (16 * m);
      else hi |= gg << (16 * (m - 4));
    }
  }
  __device__ __forceinline__ void get(int m, int& g0, int& g1) const {
    const uint32_t gg = (m < 4 ? (uint32_t)(lo >> (16 * m)) : hi >> (16 * (m - 4))) & 0xffffu;
    g0 = gg & 0xff;
    g1 = gg >> 8;
  }
};

// Stress of one voxel (sample frame) and the elastic strain and stress in
// the frame of the material table (crystal frame for ROT, sample otherwise).
struct VoxelOut {
  float sig[6];
  float sig_m[6];
  float gam_m[6];  // engineering shear
};

// Twin-variant terms of one voxel in the material frame: work = sigma : eps0_q
// and quad = eps_el : dC_q : eps_el for every variant.
template <int V, class TP>
__device__ __forceinline__ void variant_terms(TP tab, const float (&sig_m)[6], const float (&gam_m)[6],
                                              float (&work)[V], float (&quad)[V]) {
  const auto e0 = tab + 21 * (V + 1);
  // quad_q = sum_ij dC_q,ij g_i g_j over the packed upper triangle: the 21
  // products (off-diagonal ones doubled) are shared by the variants
  float gg[21];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i; j < 6; ++j) gg[sym6(i, j)] = (i == j ? 1.f : 2.f) * gam_m[i] * gam_m[j];
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const auto e0q = e0 + 6 * q;
    work[q] = sig_m[0] * e0q[0] + sig_m[1] * e0q[1] + sig_m[2] * e0q[2] +
              2.f * (sig_m[3] * e0q[3] + sig_m[4] * e0q[4] + sig_m[5] * e0q[5]);
    const auto dq = tab + 21 * (q + 1);
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 21; ++k) s += dq[k] * gg[k];
    quad[q] = s;
  }
}

// Per-grain sample-frame tables: the stress of one voxel and, for the
// phase-field pass, its variant terms. HK: the interpolation h (PF_H_LINEAR
// or PF_H_QUINTIC) as a constant, so the linear case carries no polynomial.
template <int V, bool AC, int HK>
__device__ __forceinline__ void eval_voxel(const KArgs& a, const float* tabs, const float (&e)[6],
                                           const float (&et)[V], const float (&ep)[6], int g, VoxelOut& o,
                                           float (&work)[V], float (&quad)[V]) {
  with_table(a, tabs, g, [&](auto tab) {
    Mat<V> m;
    constitutive<V>(e, et, ep, tab, HK, m);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      o.sig[c] = m.sig[c];
      o.sig_m[c] = m.sig[c];
      o.gam_m[c] = m.gam[c];
    }
    if constexpr (AC) variant_terms<V>(tab, o.sig_m, o.gam_m, work, quad);
  });
}

// variant_terms for the two voxels of a sample, the crystal table read with
// scalar loads block by block (see smem_after).
template <int V>
__device__ __forceinline__ void variant_terms_pair(ctab_t xtab, const VoxelOut (&vo)[2], float (&work)[2][V],
                                                   float (&quad)[2][V]) {
  float gg[2][21];
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = i; j < 6; ++j) gg[v][sym6(i, j)] = (i == j ? 1.f : 2.f) * vo[v].gam_m[i] * vo[v].gam_m[j];
  ctab_t t = smem_after(xtab + 21 * (V + 1), gg[1][20]);
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const ctab_t e0q = t + 6 * q;
      const float* sm = vo[v].sig_m;
      work[v][q] = sm[0] * e0q[0] + sm[1] * e0q[1] + sm[2] * e0q[2] + 2.f * (sm[3] * e0q[3] + sm[4] * e0q[4] + sm[5] * e0q[5]);
    }
  float dep = work[1][V - 1];
#pragma unroll
  for (int q = 0; q < V; ++q) {
    t = smem_after(xtab + 21 * (q + 1), dep);
    float acc[2] = {0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 21; ++k) {
#pragma unroll
      for (int v = 0; v < 2; ++v) acc[v] += t[k] * gg[v][k];
      if (k == 10) dep = acc[1];
    }
    quad[0][q] = acc[0];
    quad[1][q] = acc[1];
  }
}

// Both voxels of a packed sample: with the rotation form and scalar table
// loads the two share every table read.
// R: the grain rotations of the two voxels (rotation form), loaded by the
// caller together with the sample.
template <int V, bool ROT, bool AC, int HK>
__device__ __forceinline__ void eval_pair(const KArgs& a, const float* tabs, const float (&e)[2][6],
                                          const float (&et)[2][V], const float (&ep)[2][6], const int (&g)[2],
                                          const float (&R)[2][9], VoxelOut (&vo)[2], float (&work)[2][V],
                                          float (&quad)[2][V]) {
  if constexpr (ROT) {
    MatR<V> m[2];
    constitutive_rot_pair<V>(kernarg_xtab(), HK, e, et, ep, R, m);
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        vo[v].sig[c] = m[v].sig[c];
        vo[v].sig_m[c] = m[v].sig_c[c];
        vo[v].gam_m[c] = m[v].gam_c[c];
      }
    if constexpr (AC) variant_terms_pair<V>(kernarg_xtab(), vo, work, quad);
  } else {
#pragma unroll
    for (int v = 0; v < 2; ++v) eval_voxel<V, AC, HK>(a, tabs, e[v], et[v], ep[v], g[v], vo[v], work[v], quad[v]);
  }
}

// Chemical force of variant q: 2A f_q sum_{b != q} f_b (f_b - f_q), b over
// the other variants and the matrix f_M = 1 - sum f.
template <int V>
__device__ __forceinline__ float chem_force(float A, const float (&et)[V], float fm, int q) {
  float sm = fm * (fm - et[q]);
#pragma unroll
  for (int r = 0; r < V; ++r)
    if (r != q) sm += et[r] * (et[r] - et[q]);
  return 2.f * A * et[q] * sm;
}

// Fixed point, forward: polarisation tau = C(x):(eps - eps*) - C0:eps of
// every voxel, FP64 sum of the stress, R2C of the six components.
template <int M, int V, bool ROT, int HK>
__global__ __launch_bounds__(xthreads<M>()) __attribute__((amdgpu_waves_per_eu(kXWaves))) void k_x_fwd_ms(const KArgs a) {
  constexpr int E = XPlan<M>::E, T = M / E, ROWS = xthreads<M>() / T;
  constexpr int LROW = RowView::padded(M) + 1;
  __shared__ float2 stage[6 * ROWS * LROW];
  const int rpi = a.nz * a.ny;
  const int inst = blockIdx.x * ROWS / rpi;
  const DevState* st = a.state + inst;
  if (st->st.done) return;
  const ctab_t C0 = (ctab_t)(a.ref + (size_t)inst * kRefStride);
  const float* tabs = a.tables + (size_t)inst * a.tab_inst;
  const int t = threadIdx.x % T, p = threadIdx.x / T;
  const int nrows = a.ninst * rpi;
  const int row = blockIdx.x * ROWS + p;
  const bool valid = row < nrows;
  const size_t vs = (size_t)nrows * a.nx;
  const size_t rbase = (size_t)(valid ? row : 0) * a.nx;
  float shift[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) shift[c] = mean_shift(a, st, c);
  float fsum[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // this thread's voxels, then FP64
  GidPack<E> gids;
  gids.load(a, rbase, t, T);
#pragma unroll 1
  for (int m = 0; m < E; ++m) {
    const int k = t + T * m;
    Sample<V> s;
    load_sample<V>(a, vs, (uint32_t)(rbase + 2 * k), s);
    gids.get(m, s.g0, s.g1);
    float R[2][9];
    if constexpr (ROT) {
      load_rotation(a, s.g0, R[0]);
      load_rotation(a, s.g1, R[1]);
    }
    extrapolate_strain(a, vs, (uint32_t)(rbase + 2 * k), s.e);
    if (a.iter_mode != 0 && valid) {
      // the extrapolated first iterate, kept for the inverse pass's residual
      // (eps_out may be the oldest history field: read above, same element)
#pragma unroll
      for (int c = 0; c < 6; ++c)
        gst(reinterpret_cast<float2*>(a.eps_out + c * vs + rbase + 2 * k), s.e[c]);
    }
    float o[2][6];
    float e[2][6], ep[2][6], et[2][V];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        e[half][c] = (half ? s.e[c].y : s.e[c].x) + shift[c];
        ep[half][c] = half ? s.p[c].y : s.p[c].x;
      }
#pragma unroll
      for (int q = 0; q < V; ++q) et[half][q] = half ? s.h[q].y : s.h[q].x;
    }
    VoxelOut vo[2];
    float work[2][V], quad[2][V];
    eval_pair<V, ROT, false, HK>(a, tabs, e, et, ep, {s.g0, s.g1}, R, vo, work, quad);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      float ge[6], c0e[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) ge[c] = c < 3 ? e[half][c] : 2.f * e[half][c];
      symv6(C0, ge, c0e);
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        o[half][c] = vo[half].sig[c] - c0e[c];
        if (valid) fsum[c] += vo[half].sig[c];
      }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c)
      stage[(c * ROWS + p) * LROW + RowView::pad(k)] = make_float2(o[0][c], o[1][c]);
  }
  const size_t cs = a.cs;
  float2* dst = a.spec + (size_t)(valid ? row : 0) * a.sh;
  XTw<M, 1> tw;
  tw.load(a, t);
#pragma unroll 1
  for (int c = 0; c < 6; ++c) {
    float2* slab = stage + (c * ROWS + p) * LROW;
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = slab[RowView::pad(t + T * m)];
    r2c_one<M>(v, slab, t, valid, dst + c * cs, nyq_at(a, c, valid ? row : 0), tw);
  }
  double ssum[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) ssum[c] = (double)fsum[c];
  block_sum<6, xthreads<M>() / 64>(ssum, a.part_ms + (size_t)blockIdx.x * kQms);
}

// Phase-field update, forward: driving forces and the explicit right-hand
// side RHS_a = f_a - L dt (chem_a - mech_a) of every voxel, FP64 energy and
// mean sums, extrema of f; R2C of the V right-hand sides. With a fixed point
// over the update (PB) the part that stays fixed, f_a + L dt m mech_a, is
// kept (a separate instantiation: the store costs registers).
template <int M, int V, bool ROT, int HK, bool PB>
__global__ __launch_bounds__(xthreads<M>()) __attribute__((amdgpu_waves_per_eu(kXWaves))) void k_x_fwd_ac(const KArgs a) {
  constexpr int E = XPlan<M>::E, T = M / E, ROWS = xthreads<M>() / T;
  constexpr int LROW = RowView::padded(M) + 1;
  __shared__ float2 stage[V * ROWS * LROW];
  if (a.guard_ready && !a.state[0].st.ready) return;
  const int rpi = a.nz * a.ny;
  const int inst = blockIdx.x * ROWS / rpi;
  const float* tabs = a.tables + (size_t)inst * a.tab_inst;
  const int t = threadIdx.x % T, p = threadIdx.x / T;
  const int nrows = a.ninst * rpi;
  const int row = blockIdx.x * ROWS + p;
  const bool valid = row < nrows;
  const size_t vs = (size_t)nrows * a.nx;
  const size_t rbase = (size_t)(valid ? row : 0) * a.nx;
  float facc[kQac];  // this thread's voxels, then FP64
#pragma unroll
  for (int q = 0; q < kQac; ++q) facc[q] = 0.f;
  float mn = 3.0e38f, mx = -3.0e38f;
  GidPack<E> gids;
  gids.load(a, rbase, t, T);
#pragma unroll 1
  for (int m = 0; m < E; ++m) {
    const int k = t + T * m;
    const int x0 = 2 * k;
    Sample<V> s;
    load_sample<V>(a, vs, (uint32_t)(rbase + x0), s);
    gids.get(m, s.g0, s.g1);
    float R[2][9];
    if constexpr (ROT) {
      load_rotation(a, s.g0, R[0]);
      load_rotation(a, s.g1, R[1]);
    }
    float o[2][V];
    float e2[2][6], ep2[2][6], et2[2][V];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        e2[half][c] = half ? s.e[c].y : s.e[c].x;
        ep2[half][c] = half ? s.p[c].y : s.p[c].x;
      }
#pragma unroll
      for (int q = 0; q < V; ++q) et2[half][q] = half ? s.h[q].y : s.h[q].x;
    }
    VoxelOut vo2[2];
    float work2[2][V], quad2[2][V];
    eval_pair<V, ROT, true, HK>(a, tabs, e2, et2, ep2, {s.g0, s.g1}, R, vo2, work2, quad2);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const float (&e)[6] = e2[half];
      const float (&et)[V] = et2[half];
      const VoxelOut& vo = vo2[half];
      const float (&work)[V] = work2[half];
      const float (&quad)[V] = quad2[half];
      float fm = 1.f;
#pragma unroll
      for (int q = 0; q < V; ++q) fm -= et[q];
      // double well over the variants and the matrix: sum_{a<b} f_a^2 f_b^2
      float fdw = 0.f;
#pragma unroll
      for (int q = 0; q < V; ++q) {
        fdw += et[q] * et[q] * fm * fm;
#pragma unroll
        for (int r = q + 1; r < V; ++r) fdw += et[q] * et[q] * et[r] * et[r];
      }
      float fme = 0.f;
#pragma unroll
      for (int c = 0; c < 6; ++c) fme += vo.sig_m[c] * vo.gam_m[c];
#pragma unroll
      for (int q = 0; q < V; ++q) {
        // mech_a = h'(f_a) [sigma : eps0_a - 1/2 eps_el : dC_a : eps_el]
        const float mech = dh_of(et[q], HK) * (work[q] - 0.5f * quad[q]);
        o[half][q] = et[q] - a.LDt * (chem_force<V>(a.A, et, fm, q) - mech);
        if (PB && valid) {
          const size_t vox = rbase + x0 + half;
          const float mb = a.mob ? a.mob[vox] : 1.f;
          a.pf_base[q * vs + vox] = et[q] + mb * a.LDt * mech;
        }
      }
      if (a.mob) {
        // relative mobility m: the local forces scaled by m, the gradient
        // term's explicit part L dt (m - 1) G(f^n) (the implicit part uses L)
        const size_t vox = rbase + x0 + half;
        const float mb = a.mob[vox];
#pragma unroll
        for (int q = 0; q < V; ++q)
          o[half][q] = et[q] + mb * (o[half][q] - et[q]) + a.LDt * (mb - 1.f) * a.lapf[q * vs + vox];
      }
      if (valid) {
        facc[0] += fdw;
        facc[1] += 0.5f * fme;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          facc[2 + c] += vo.sig[c];
          facc[8 + c] += e[c];
        }
#pragma unroll
        for (int q = 0; q < V; ++q) {
          facc[14 + q] += et[q];
          mn = fminf(mn, et[q]);
          mx = fmaxf(mx, et[q]);
        }
        if (a.save_stress) {
#pragma unroll
          for (int c = 0; c < 6; ++c) a.sig[c * vs + rbase + x0 + half] = vo.sig[c];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < V; ++q)
      stage[(q * ROWS + p) * LROW + RowView::pad(k)] = make_float2(o[0][q], o[1][q]);
  }
  const size_t cs = a.cs;
  float2* dst = a.spec + (size_t)(valid ? row : 0) * a.sh;
  XTw<M, 1> tw;
  tw.load(a, t);
#pragma unroll 1
  for (int q = 0; q < V; ++q) {
    float2* slab = stage + (q * ROWS + p) * LROW;
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = slab[RowView::pad(t + T * m)];
    r2c_one<M>(v, slab, t, valid, dst + q * cs, nyq_at(a, q, valid ? row : 0), tw);
  }
  double acc[kQac];
#pragma unroll
  for (int q = 0; q < kQac; ++q) acc[q] = (double)facc[q];
  block_sum<kQac, xthreads<M>() / 64>(acc, a.part_ac + (size_t)blockIdx.x * kQac);
  block_minmax<xthreads<M>() / 64>(mn, mx, a.part_mm + 2 * (size_t)blockIdx.x);
}


// Fixed point over the update, forward pass of a further solve: the
// right-hand side b_a - L dt m chem_a(f^{i-1}) (+ L dt (m - 1) G(f^{i-1})
// with a mobility field) from the kept base b_a = f^n_a + L dt m mech_a,
// R2C of the V components. The reductions of the step stay those of its
// first pass.
template <int M, int V>
__global__ __launch_bounds__(xthreads<M>()) void k_x_fwd_pc(const KArgs a) {
  constexpr int E = XPlan<M>::E, T = M / E, ROWS = xthreads<M>() / T;
  constexpr int LROW = RowView::padded(M) + 1;
  __shared__ float2 stage[V * ROWS * LROW];
  const int t = threadIdx.x % T, p = threadIdx.x / T;
  const int nrows = a.ninst * a.nz * a.ny;
  const int row = blockIdx.x * ROWS + p;
  const bool valid = row < nrows;
  const size_t vs = (size_t)nrows * a.nx;
  const size_t rbase = (size_t)(valid ? row : 0) * a.nx;
#pragma unroll 1
  for (int m = 0; m < E; ++m) {
    const int k = t + T * m;
    const size_t vox = rbase + 2 * k;
    float2 f[V], b[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
      f[q] = *reinterpret_cast<const float2*>(a.eta + q * vs + vox);
      b[q] = *reinterpret_cast<const float2*>(a.pf_base + q * vs + vox);
    }
    float o[2][V];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      float et[V];
      float fm = 1.f;
#pragma unroll
      for (int q = 0; q < V; ++q) {
        et[q] = half ? f[q].y : f[q].x;
        fm -= et[q];
      }
#pragma unroll
      for (int q = 0; q < V; ++q) o[half][q] = (half ? b[q].y : b[q].x) - a.LDt * chem_force<V>(a.A, et, fm, q);
    }
    if (a.mob) {
      const float2 mb = *reinterpret_cast<const float2*>(a.mob + vox);
#pragma unroll
      for (int q = 0; q < V; ++q) {
        const float2 g = *reinterpret_cast<const float2*>(a.lapf + q * vs + vox);
        const float b0 = b[q].x, b1 = b[q].y;
        o[0][q] = b0 + mb.x * (o[0][q] - b0) + a.LDt * (mb.x - 1.f) * g.x;
        o[1][q] = b1 + mb.y * (o[1][q] - b1) + a.LDt * (mb.y - 1.f) * g.y;
      }
    }
#pragma unroll
    for (int q = 0; q < V; ++q)
      stage[(q * ROWS + p) * LROW + RowView::pad(k)] = make_float2(o[0][q], o[1][q]);
  }
  const size_t cs = a.cs;
  float2* dst = a.spec + (size_t)(valid ? row : 0) * a.sh;
  XTw<M, 1> tw;
  tw.load(a, t);
#pragma unroll 1
  for (int q = 0; q < V; ++q) {
    float2* slab = stage + (q * ROWS + p) * LROW;
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = slab[RowView::pad(t + T * m)];
    r2c_one<M>(v, slab, t, valid, dst + q * cs, nyq_at(a, q, valid ? row : 0), tw);
  }
}

#if PF_NV <= 3
// Homogeneous spectral path, forward: R2C of f_a (components 0..V-1) and of
// f_a - L dt chem_a (components V..2V-1; with resid, L dt chem_a: the force
// of one state, as the autotuner times the z pass); FP64 double-well and mean
// sums, extrema of f. The elastic force is applied per wavevector in the z
// pass.
template <int M, int V>
__global__ __launch_bounds__(xthreads<M>()) void k_x_fwd_kh(const KArgs a, int resid) {
  constexpr int E = XPlan<M>::E, T = M / E, ROWS = xthreads<M>() / T;
  constexpr int LROW = RowView::padded(M) + 1;
  __shared__ float2 stage[2 * V * ROWS * LROW];
  const int t = threadIdx.x % T, p = threadIdx.x / T;
  const int nrows = a.ninst * a.nz * a.ny;
  const int row = blockIdx.x * ROWS + p;
  const bool valid = row < nrows;
  const size_t vs = (size_t)nrows * a.nx;
  const size_t rbase = (size_t)(valid ? row : 0) * a.nx;
  float facc[1 + V];
#pragma unroll
  for (int q = 0; q <= V; ++q) facc[q] = 0.f;
  float mn = 3.0e38f, mx = -3.0e38f;
#pragma unroll 1
  for (int m = 0; m < E; ++m) {
    const int k = t + T * m;
    float2 h[V];
#pragma unroll
    for (int q = 0; q < V; ++q)
      h[q] = valid ? *reinterpret_cast<const float2*>(a.eta + q * vs + rbase + 2 * k) : make_float2(0.f, 0.f);
    float o[2][V];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      float et[V];
#pragma unroll
      for (int q = 0; q < V; ++q) et[q] = half ? h[q].y : h[q].x;
      float fm = 1.f;
#pragma unroll
      for (int q = 0; q < V; ++q) fm -= et[q];
      float fdw = 0.f;
#pragma unroll
      for (int q = 0; q < V; ++q) {
        fdw += et[q] * et[q] * fm * fm;
#pragma unroll
        for (int r = q + 1; r < V; ++r) fdw += et[q] * et[q] * et[r] * et[r];
      }
#pragma unroll
      for (int q = 0; q < V; ++q) {
        const float lc = a.LDt * chem_force<V>(a.A, et, fm, q);
        o[half][q] = resid ? lc : et[q] - lc;
      }
      if (valid) {
        facc[0] += fdw;
#pragma unroll
        for (int q = 0; q < V; ++q) {
          facc[1 + q] += et[q];
          mn = fminf(mn, et[q]);
          mx = fmaxf(mx, et[q]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < V; ++q) {
      stage[(q * ROWS + p) * LROW + RowView::pad(k)] = h[q];
      stage[((V + q) * ROWS + p) * LROW + RowView::pad(k)] = make_float2(o[0][q], o[1][q]);
    }
  }
  const size_t cs = a.cs;
  float2* dst = a.spec + (size_t)(valid ? row : 0) * a.sh;
  XTw<M, 1> tw;
  tw.load(a, t);
#pragma unroll 1
  for (int c = 0; c < 2 * V; ++c) {
    float2* slab = stage + (c * ROWS + p) * LROW;
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = slab[RowView::pad(t + T * m)];
    r2c_one<M>(v, slab, t, valid, dst + c * cs, nyq_at(a, c, valid ? row : 0), tw);
  }
  double acc[kQac];
#pragma unroll
  for (int q = 0; q < kQac; ++q) acc[q] = 0.0;
  acc[0] = (double)facc[0];
#pragma unroll
  for (int q = 0; q < V; ++q) acc[14 + q] = (double)facc[1 + q];
  block_sum<kQac, xthreads<M>() / 64>(acc, a.part_ac + (size_t)blockIdx.x * kQac);
  block_minmax<xthreads<M>() / 64>(mn, mx, a.part_mm + 2 * (size_t)blockIdx.x);
}

// Residual of a macro step of S plain steps from f0 (prev) to f1 (the
// current order parameter), forward x pass. Summing S plain steps (local
// force explicit, gradient force implicit: Sec. 3, eqs. (19)-(20)) and taking
// both sums by the trapezoid rule with the end correction of a left (right)
// Riemann sum, with p = (S+1)/2, m = (S-1)/2:
//   r = f1 - f0 + L dt [p chem(f0) + m chem(f1)] - L dt [p mech(f0) + m mech(f1)]
//       + L dt G (m f0 + p f1).
// mech is affine in f with one stiffness and linear h, so its two terms are
// S mech(u) with u = (p f0 + m f1) / S. R2C of u (components 0..V-1, whose
// FP64 sums feed the mixed condition of the z pass), of L dt (p chem(f0) +
// m chem(f1)) / S (V..2V-1) and of w = (m f0 + p f1) / S (2V..3V-1); the z
// pass (mode 2) forms L dt [chem part / S + G w - mech(u)], and the inverse
// pass r = f1 - f0 + S times that. u and the chemical part are staged
// together; w, which needs no other component, row by row after them.
template <int M, int V>
__global__ __launch_bounds__(xthreads<M>()) void k_x_fwd_ct(const KArgs a, const float* __restrict__ prev,
                                                           float S) {
  constexpr int E = XPlan<M>::E, T = M / E, ROWS = xthreads<M>() / T;
  constexpr int LROW = RowView::padded(M) + 1;
  __shared__ float2 stage[2 * V * ROWS * LROW];
  const int t = threadIdx.x % T, p = threadIdx.x / T;
  const int nrows = a.ninst * a.nz * a.ny;
  const int row = blockIdx.x * ROWS + p;
  const bool valid = row < nrows;
  const size_t vs = (size_t)nrows * a.nx;
  const size_t rbase = (size_t)(valid ? row : 0) * a.nx;
  const float wp = 0.5f * (S + 1.f) / S, wm = 0.5f * (S - 1.f) / S;
  float facc[V];
#pragma unroll
  for (int q = 0; q < V; ++q) facc[q] = 0.f;
#pragma unroll 1
  for (int m = 0; m < E; ++m) {
    const int k = t + T * m;
    float2 h0[V], h1[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const size_t off = q * vs + rbase + 2 * k;
      h0[q] = valid ? *reinterpret_cast<const float2*>(prev + off) : make_float2(0.f, 0.f);
      h1[q] = valid ? *reinterpret_cast<const float2*>(a.eta + off) : make_float2(0.f, 0.f);
    }
    float o[2][2][V];  // [half][u, chemical part][q]
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      float e0[V], e1[V];
      float fm0 = 1.f, fm1 = 1.f;
#pragma unroll
      for (int q = 0; q < V; ++q) {
        e0[q] = half ? h0[q].y : h0[q].x;
        e1[q] = half ? h1[q].y : h1[q].x;
        fm0 -= e0[q];
        fm1 -= e1[q];
      }
#pragma unroll
      for (int q = 0; q < V; ++q) {
        o[half][0][q] = wp * e0[q] + wm * e1[q];
        o[half][1][q] = a.LDt * (wp * chem_force<V>(a.A, e0, fm0, q) + wm * chem_force<V>(a.A, e1, fm1, q));
        if (valid) facc[q] += o[half][0][q];
      }
    }
#pragma unroll
    for (int q = 0; q < V; ++q) {
      stage[(q * ROWS + p) * LROW + RowView::pad(k)] = make_float2(o[0][0][q], o[1][0][q]);
      stage[((V + q) * ROWS + p) * LROW + RowView::pad(k)] = make_float2(o[0][1][q], o[1][1][q]);
    }
  }
  const size_t cs = a.cs;
  float2* dst = a.spec + (size_t)(valid ? row : 0) * a.sh;
  XTw<M, 1> tw;
  tw.load(a, t);
#pragma unroll 1
  for (int c = 0; c < 2 * V; ++c) {
    float2* slab = stage + (c * ROWS + p) * LROW;
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = slab[RowView::pad(t + T * m)];
    r2c_one<M>(v, slab, t, valid, dst + c * cs, nyq_at(a, c, valid ? row : 0), tw);
  }
#pragma unroll 1
  for (int q = 0; q < V; ++q) {
    // w of variant q straight from the two fields, through this row's first slab
    float2* slab = stage + p * LROW;
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const size_t off = q * vs + rbase + 2 * (t + T * m);
      const float2 x0 = valid ? *reinterpret_cast<const float2*>(prev + off) : make_float2(0.f, 0.f);
      const float2 x1 = valid ? *reinterpret_cast<const float2*>(a.eta + off) : make_float2(0.f, 0.f);
      v[m] = make_float2(wm * x0.x + wp * x1.x, wm * x0.y + wp * x1.y);
    }
    r2c_one<M>(v, slab, t, valid, dst + (2 * V + q) * cs, nyq_at(a, 2 * V + q, valid ? row : 0), tw);
  }
  double acc[kQac];
#pragma unroll
  for (int q = 0; q < kQac; ++q) acc[q] = 0.0;
#pragma unroll
  for (int q = 0; q < V; ++q) acc[14 + q] = (double)facc[q];
  block_sum<kQac, xthreads<M>() / 64>(acc, a.part_ac + (size_t)blockIdx.x * kQac);
}
#endif
}  // namespace pft

#define PF_CAT2(a, b) a##b
#define PF_CAT(a, b) PF_CAT2(a, b)

namespace pfl {
using namespace pft;

#define PF_SWITCH_M_LOCAL(nx, BODY)                   \
  switch ((nx) / 2) {                                  \
    case 16: { constexpr int M = 16; BODY; } break;   \
    case 24: { constexpr int M = 24; BODY; } break;   \
    case 32: { constexpr int M = 32; BODY; } break;   \
    case 48: { constexpr int M = 48; BODY; } break;   \
    case 64: { constexpr int M = 64; BODY; } break;   \
    case 96: { constexpr int M = 96; BODY; } break;   \
    case 128: { constexpr int M = 128; BODY; } break; \
    case 192: { constexpr int M = 192; BODY; } break; \
    case 256: { constexpr int M = 256; BODY; } break; \
    default: return hipErrorInvalidValue;              \
  }

#define PF_LAUNCH_X(KERNEL, ...)                                                                    \
  do {                                                                                              \
    const dim3 grid(x_blocks(a));                                                                   \
    const bool q = a.h_kind == 1;                                                                   \
    if (a.rot && q) {                                                                               \
      PF_SWITCH_M_LOCAL(a.nx, (KERNEL<M, PF_NV, true, 1 __VA_ARGS__><<<grid, xthreads<M>(), 0, s>>>(a)));   \
    } else if (a.rot) {                                                                             \
      PF_SWITCH_M_LOCAL(a.nx, (KERNEL<M, PF_NV, true, 0 __VA_ARGS__><<<grid, xthreads<M>(), 0, s>>>(a)));   \
    } else if (q) {                                                                                 \
      PF_SWITCH_M_LOCAL(a.nx, (KERNEL<M, PF_NV, false, 1 __VA_ARGS__><<<grid, xthreads<M>(), 0, s>>>(a)));  \
    } else {                                                                                        \
      PF_SWITCH_M_LOCAL(a.nx, (KERNEL<M, PF_NV, false, 0 __VA_ARGS__><<<grid, xthreads<M>(), 0, s>>>(a)));  \
    }                                                                                               \
  } while (0)

hipError_t PF_CAT(ms_x_forward_v, PF_NV)(const KArgs& a, hipStream_t s) {
  PF_LAUNCH_X(k_x_fwd_ms);
  return hipGetLastError();
}

#if PF_NV <= 3
hipError_t PF_CAT(kh_x_forward_v, PF_NV)(const KArgs& a, int resid, hipStream_t s) {
  const dim3 grid(x_blocks(a));
  PF_SWITCH_M_LOCAL(a.nx, (k_x_fwd_kh<M, PF_NV><<<grid, xthreads<M>(), 0, s>>>(a, resid)));
  return hipGetLastError();
}

hipError_t PF_CAT(ct_x_forward_v, PF_NV)(const KArgs& a, const float* prev, int n_steps, hipStream_t s) {
  const dim3 grid(x_blocks(a));
  PF_SWITCH_M_LOCAL(a.nx, (k_x_fwd_ct<M, PF_NV><<<grid, xthreads<M>(), 0, s>>>(a, prev, (float)n_steps)));
  return hipGetLastError();
}
#endif

hipError_t PF_CAT(ac_x_forward_v, PF_NV)(const KArgs& a, hipStream_t s) {
  if (a.pf_base) {
    PF_LAUNCH_X(k_x_fwd_ac, , true);
  } else {
    PF_LAUNCH_X(k_x_fwd_ac, , false);
  }
  return hipGetLastError();
}

hipError_t PF_CAT(pc_x_forward_v, PF_NV)(const KArgs& a, hipStream_t s) {
  const dim3 grid(x_blocks(a));
  PF_SWITCH_M_LOCAL(a.nx, (k_x_fwd_pc<M, PF_NV><<<grid, xthreads<M>(), 0, s>>>(a)));
  return hipGetLastError();
}

}  // namespace pfl
