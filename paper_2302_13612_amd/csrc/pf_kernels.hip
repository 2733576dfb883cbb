// HIP kernels of the FFT phase-field twin step (gfx950).
//
// A 3D real-to-complex transform is three passes over HBM:
//   x: contiguous rows; a real row of length nx is packed into nx/2 complex
//      samples, transformed, and split into nx/2+1 coefficients. The x pass
//      fuses the per-voxel physics: the constitutive law (polarisation of the
//      fixed point) before the forward transform, the strain update after the
//      inverse one; and the driving forces of the phase-field update.
//   y: columns of 16 consecutive kx (128-byte runs), in place.
//   z: columns like y; the forward transform, the per-wavevector operator and
//      the inverse transform run in one kernel with the pencil in registers,
//      so the spectrum makes one round trip through HBM for the z stage.
// Reductions are FP64 partial sums per block followed by a one-block
// finalize in a fixed order (deterministic).
#include "pf_common.hpp"

namespace pft {

// -------------------------------------------------------------- x kernels
// Fixed point, inverse: new strain field from the six spectra, FP64 sums of
// the squared change and the squared new strain (full tensor norm).
template <int M>
__global__ __launch_bounds__(xthreads<M>()) void k_x_inv_ms(const KArgs a) {
  constexpr int E = XPlan<M>::E, T = M / E, ROWS = xthreads<M>() / T;
  constexpr int LROW = RowView::padded(M) + 1;
  __shared__ float2 lds[ROWS * LROW];
  const int rpi = a.nz * a.ny;
  const int inst = blockIdx.x * ROWS / rpi;
  const DevState* st = a.state + inst;
  if (st->st.done) return;
  const int t = threadIdx.x % T, p = threadIdx.x / T;
  const int nrows = a.ninst * rpi;
  const int row = blockIdx.x * ROWS + p;
  const bool valid = row < nrows;
  const int nx = a.nx;
  const size_t vs = (size_t)nrows * nx;
  const size_t rbase = (size_t)(valid ? row : 0) * nx;
  const size_t cs = a.cs;
  const size_t roff = (size_t)(valid ? row : 0) * a.sh;
  const size_t rowv = valid ? row : 0;
  double acc[2] = {0.0, 0.0};
  // component c+1's spectral row is fetched while component c is transformed
  RowFetch<M> cur, nxt;
  c2r_fetch<M>(cur, t, valid, a.spec + roff, nyq_at(a, 0, rowv));
  XTw<M, -1> tw;
  tw.load(a, t);
  // the iterate this iteration started from: the stored strain, or on the
  // first iteration of a step the extrapolated one the forward pass wrote
  const float* prev = a.iter_mode != 0 ? a.eps_out : a.eps;
  float2 old_c[E];
#pragma unroll 1
  for (int c = 0; c < 6; ++c) {
    if (c + 1 < 6) c2r_fetch<M>(nxt, t, valid, a.spec + (c + 1) * cs + roff, nyq_at(a, c + 1, rowv));
    // this component's old iterate, in flight while its row is transformed
    // (fetching it one component ahead costs registers and gains nothing)
#pragma unroll
    for (int m = 0; m < E; ++m)
      old_c[m] = valid ? gld(reinterpret_cast<const float2*>(prev + c * vs + rbase + 2 * (t + T * m)))
                       : make_float2(0.f, 0.f);
    const float shift = (float)(st->ebar_cur[c] - st->ebar_base[c]);
    const float w = c < 3 ? 1.f : 2.f;
    float2 v[E];
    c2r_from_regs<M>(v, cur, lds + p * LROW, t, tw);
    float dsum = 0.f, nsum = 0.f;
    if (valid) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const size_t off = c * vs + rbase + 2 * (t + T * m);
        const float2 old = old_c[m];
        const float dx0 = v[m].x - (old.x + shift), dx1 = v[m].y - (old.y + shift);
        dsum += dx0 * dx0 + dx1 * dx1;
        nsum += v[m].x * v[m].x + v[m].y * v[m].y;
        // on a first iteration the output is the field read above as the old iterate
        gst(reinterpret_cast<float2*>(a.eps_out + off), v[m]);
      }
    }
    acc[0] += (double)(w * dsum);
    acc[1] += (double)(w * nsum);
    cur = nxt;
  }
  block_sum<2, xthreads<M>() / 64>(acc, a.part_res + (size_t)blockIdx.x * kQres);
}

// Phase-field update, inverse: new order parameters, count of non-finite
// values; with a fixed point over the update also the per-block max change
// max |f^i - f^{i-1}| against the values overwritten.
template <int M>
__global__ __launch_bounds__(xthreads<M>()) void k_x_inv_ac(const KArgs a) {
  constexpr int E = XPlan<M>::E, T = M / E, ROWS = xthreads<M>() / T;
  constexpr int LROW = RowView::padded(M) + 1;
  __shared__ float2 lds[ROWS * LROW];
  if (a.guard_ready && !a.state[0].st.ready) return;
  const int t = threadIdx.x % T, p = threadIdx.x / T;
  const int nrows = a.ninst * a.nz * a.ny;
  const int row = blockIdx.x * ROWS + p;
  const bool valid = row < nrows;
  const size_t vs = (size_t)nrows * a.nx;
  const size_t rbase = (size_t)(valid ? row : 0) * a.nx;
  const size_t cs = a.cs;
  const size_t roff = (size_t)(valid ? row : 0) * a.sh;
  const size_t rowv = valid ? row : 0;
  double bad[1] = {0.0};
  float dmax = 0.f;
  RowFetch<M> cur, nxt;
  c2r_fetch<M>(cur, t, valid, a.spec + roff, nyq_at(a, 0, rowv));
  XTw<M, -1> tw;
  tw.load(a, t);
  // components 0..nv-1: the new f; with a mobility field also nv..2nv-1:
  // the gradient force of the new f, kept for the next step
  const int nc = a.lapf ? 2 * a.nv : a.nv;
#pragma unroll 1
  for (int q = 0; q < nc; ++q) {
    if (q + 1 < nc) c2r_fetch<M>(nxt, t, valid, a.spec + (q + 1) * cs + roff, nyq_at(a, q + 1, rowv));
    float2 v[E];
    c2r_from_regs<M>(v, cur, lds + p * LROW, t, tw);
    if (valid) {
      float* dst = q < a.nv ? a.eta + q * vs : a.lapf + (q - a.nv) * vs;
      if (a.part_pc && q < a.nv) {
        float2 old[E];
#pragma unroll
        for (int m = 0; m < E; ++m) old[m] = gld(reinterpret_cast<const float2*>(dst + rbase + 2 * (t + T * m)));
#pragma unroll
        for (int m = 0; m < E; ++m)
          dmax = fmaxf(dmax, fmaxf(fabsf(v[m].x - old[m].x), fabsf(v[m].y - old[m].y)));
      }
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int x0 = 2 * (t + T * m);
        if (q < a.nv && (!isfinite(v[m].x) || !isfinite(v[m].y))) bad[0] += 1.0;
        gst(reinterpret_cast<float2*>(dst + rbase + x0), v[m]);
      }
    }
    cur = nxt;
  }
  block_sum<1, xthreads<M>() / 64>(bad, a.part_res + (size_t)blockIdx.x * kQres);
  if (a.part_pc) block_minmax<xthreads<M>() / 64>(0.f, dmax, a.part_pc + 2 * (size_t)blockIdx.x);
}

// Plain transforms of caller fields (checking the passes).
template <int M>
__global__ __launch_bounds__(xthreads<M>()) void k_x_fwd_raw(const KArgs a, const float* __restrict__ real) {
  constexpr int E = XPlan<M>::E, T = M / E, ROWS = xthreads<M>() / T;
  constexpr int LROW = RowView::padded(M) + 1;
  __shared__ float2 lds[ROWS * LROW];
  const int t = threadIdx.x % T, p = threadIdx.x / T;
  const int nrows = a.ninst * a.nz * a.ny;
  const int row = blockIdx.x * ROWS + p;
  const bool valid = row < nrows;
  const int comp = blockIdx.y;
  const size_t vs = (size_t)nrows * a.nx;
  const size_t rbase = (size_t)(valid ? row : 0) * a.nx;
  float2 v[1][E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int x0 = 2 * (t + T * m);
    v[0][m] = valid ? *reinterpret_cast<const float2*>(real + comp * vs + rbase + x0) : make_float2(0.f, 0.f);
  }
  const size_t cs = a.cs;
  r2c_rows<M, 1>(v, lds + p * LROW, t, valid, a.spec + comp * cs, (size_t)(valid ? row : 0) * a.sh, cs,
                 nyq_at(a, comp, valid ? row : 0), a.tw_xh, a.tw_x);
}

template <int M>
__global__ __launch_bounds__(xthreads<M>()) void k_x_inv_raw(const KArgs a, float* __restrict__ real, float scale) {
  constexpr int E = XPlan<M>::E, T = M / E, ROWS = xthreads<M>() / T;
  constexpr int LROW = RowView::padded(M) + 1;
  __shared__ float2 lds[ROWS * LROW];
  const int t = threadIdx.x % T, p = threadIdx.x / T;
  const int nrows = a.ninst * a.nz * a.ny;
  const int row = blockIdx.x * ROWS + p;
  const bool valid = row < nrows;
  const int comp = blockIdx.y;
  const size_t vs = (size_t)nrows * a.nx;
  const size_t rbase = (size_t)(valid ? row : 0) * a.nx;
  const size_t cs = a.cs;
  XTw<M, -1> tw;
  tw.load(a, t);
  float2 v[E];
  c2r_row<M>(v, lds + p * LROW, t, valid, a.spec + comp * cs + (size_t)(valid ? row : 0) * a.sh,
             nyq_at(a, comp, valid ? row : 0), tw);
  if (valid) {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int x0 = 2 * (t + T * m);
      *reinterpret_cast<float2*>(real + comp * vs + rbase + x0) = cscale(v[m], scale);
    }
  }
}

// ------------------------------------------------------------ y and z passes
// y: columns of C consecutive kx at one z, in place. grid (tiles, nz, ncomp),
// where with a Nyquist plane the last x index holds the plane: its block y
// takes the C consecutive z (all of one instance: nz is a multiple of C) whose
// y pencils, contiguous in the plane, are its C columns; the blocks past the
// plane's z range have nothing to do. C (8 or 16) is the group's tuned tile.
template <int N, int K>
using PV = typename PlanV<N, K>::P;
template <int N, int K, int C>
constexpr int col_threads() { return C * (N / PV<N, K>::E); }

template <int N, int DIR, int C, int K>
__global__ __launch_bounds__((col_threads<N, K, C>())) void k_y(const KArgs a) {
  using P = PV<N, K>;
  constexpr int E = P::E, T = N / E;
  __shared__ float2 lds[N * C];
  const int cc = threadIdx.x % C, t = threadIdx.x / C;
  const int comp = blockIdx.z;
  const int nzt = a.nz * a.ninst;                // z over all instances
  const bool plane = !a.nq_row && (int)blockIdx.x == (a.ncol + C - 1) / C;
  int z0;                                        // first z of the block
  bool valid;
  float2* col;
  size_t es;                                     // stride between consecutive ky
  if (!plane) {
    const int kx = blockIdx.x * C + cc;
    z0 = blockIdx.y;
    valid = kx < a.ncol;
    es = a.sh;
    col = a.spec + comp * a.cs + (size_t)z0 * a.ny * a.sh + (valid ? kx : 0);
  } else {
    z0 = blockIdx.y * C;
    if (z0 >= nzt) return;                       // the whole block: no barrier skipped
    valid = true;
    es = 1;
    col = a.spec + comp * a.cs + a.nqo + (size_t)(z0 + cc) * a.ny;
  }
  // transforms of a fixed-point iteration are skipped for a converged instance
  if (a.skip_done && a.state[z0 / a.nz].st.done) return;
  if (a.guard_ready && !a.state[0].st.ready) return;
  float2 v[E];
#pragma unroll
  // plain loads (measured faster here than with the hint), streaming stores
  for (int m = 0; m < E; ++m) v[m] = valid ? col[(size_t)(t + T * m) * es] : make_float2(0.f, 0.f);
  fft_pencil<N, DIR, P>(v, ColView<C>{lds + cc}, t, a.tw_y);
  if (valid) {
#pragma unroll
    for (int m = 0; m < E; ++m) gst(col + (size_t)(t + T * m) * es, v[m]);
  }
}

// Signed index of coefficient k on an axis of length n (Nyquist -> -n/2).
__device__ __forceinline__ int signed_k(int k, int n) { return k < n / 2 ? k : k - n; }

// Gradient-energy symbols of one column (kx, ky) of variant q as quadratics
// in the z wave number: the semi-implicit denominator 1 + 2 L dt xi.K.xi and
// the Parseval symbol (kappa |xi|^2 up to the host's kappa factor, or
// xi.K.xi from the instance's tables). A wave number at its Nyquist index
// enters the diagonal terms only (the cross terms are odd in it).
// GK: the tables are given (a.gk); otherwise the isotropic per-axis factors.
template <bool GK>
struct GradSym {
  float d0, d1, d2;  // den - 1 = d0 + d1 kcz + d2 kz^2
  float g0, g1, g2;  // symbol  = g0 + g1 kcz + g2 kz^2
  GradSym() = default;
  __device__ __forceinline__ GradSym(const KArgs& a, int inst, int q, int kx, int sy) {
    const float fx = (float)kx * (float)kx, fy = (float)sy * (float)sy;
    if constexpr (!GK) {
      d0 = a.ax * fx + a.ay * fy, d1 = 0.f, d2 = a.az;
      g0 = (float)a.gx * fx + (float)a.gy * fy, g1 = 0.f, g2 = (float)a.gz;
      return;
    }
    const ctab_t t = (ctab_t)(a.gk + (size_t)inst * kGkStride + 12 * q);
    const float cx = kx == a.nx / 2 ? 0.f : (float)kx, cy = 2 * sy == -a.ny ? 0.f : (float)sy;
    d0 = t[0] * fx + t[1] * fy + t[5] * cx * cy, d1 = t[3] * cy + t[4] * cx, d2 = t[2];
    g0 = t[6] * fx + t[7] * fy + t[11] * cx * cy, g1 = t[9] * cy + t[10] * cx, g2 = t[8];
  }
  // cz: the z wave number for the cross terms (0 at the Nyquist index)
  __device__ __forceinline__ float den(float cz, float fz) const {
    if constexpr (GK) return 1.f + d0 + cz * d1 + d2 * fz;
    return 1.f + d0 + d2 * fz;
  }
  __device__ __forceinline__ float sym(float cz, float fz) const {
    if constexpr (GK) return g0 + cz * g1 + g2 * fz;
    return g0 + g2 * fz;
  }
};

__device__ __forceinline__ float cross_k(int sz, int n) { return 2 * sz == -n ? 0.f : (float)sz; }

// Logical block index that gives consecutive ids to the blocks the hardware
// deals to one XCD (blocks go round-robin to the 8 XCDs), so neighbouring
// column tiles that share 128-byte lines run under the same L2.
__device__ __forceinline__ int xcd_logical(int b, int nb) {
  const int q = nb / 8, r = nb % 8;
  const int x = b % 8, i = b / 8;
  return x * q + (x < r ? x : r) + i;
}

// Acoustic tensor K_ik(xi) = C0_ijkl xi_j xi_l of a column (xi_x, xi_y fixed,
// xi_z = c varying) as K0 + c (K1 + c K2); entries in the order 00 01 02 11 12 22.
__device__ __forceinline__ void acoustic_parts(ctab_t C0, float x0, float x1, float (&K0)[6],
                                               float (&K1)[6], float (&K2)[6]) {
  constexpr int VI[3][3] = {{0, 5, 4}, {5, 1, 3}, {4, 3, 2}};
  constexpr int II[6] = {0, 0, 0, 1, 1, 2}, KK[6] = {0, 1, 2, 1, 2, 2};
  const float xi[2] = {x0, x1};
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int i = II[e], k = KK[e];
    float k0 = 0.f, k1 = 0.f;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
      for (int l = 0; l < 2; ++l) k0 += C0[sym6(VI[i][j], VI[k][l])] * xi[j] * xi[l];
      k1 += (C0[sym6(VI[i][j], VI[k][2])] + C0[sym6(VI[i][2], VI[k][j])]) * xi[j];
    }
    K0[e] = k0;
    K1[e] = k1;
    K2[e] = C0[sym6(VI[i][2], VI[k][2])];
  }
}

// Green's operator step of the fixed point at one wavevector xi (any scale:
// the operator is homogeneous of degree 0): eps = -Gamma0 : tau / N with
// Gamma0 : tau = sym(xi (x) K(xi)^{-1} (tau xi)); the prescribed mean at
// xi = 0; the reference compliance at the ambiguous Nyquist wavevectors.
// Wavevector with a Nyquist index and another non-zero, non-Nyquist index:
// the continuous operator is not Hermitian-consistent there.
__device__ __forceinline__ bool ambiguous_nyquist(const KArgs& a, int kx, int ky, int kz) {
  const bool nqx = kx == a.nx / 2, nqy = ky == a.ny / 2, nqz = kz == a.nz / 2;
  const bool otx = kx != 0 && !nqx, oty = ky != 0 && !nqy, otz = kz != 0 && !nqz;
  return (nqx || nqy || nqz) && (otx || oty || otz);
}

// ebar: the mean strain of the next iterate (read at xi = 0 only)
__device__ __forceinline__ void green_apply(const KArgs& a, const double* ebar, ctab_t S0, int kx, int ky,
                                            int kz, const float (&xi)[3], const float (&K)[6],
                                            float2 (&tau)[6]) {
  if (kx == 0 && ky == 0 && kz == 0) {
#pragma unroll
    for (int c = 0; c < 6; ++c) tau[c] = make_float2((float)ebar[c], 0.f);
    return;
  }
  const float s = a.inv_ntot;
  if (ambiguous_nyquist(a, kx, ky, kz)) {
    float2 o[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        acc.x += S0[6 * i + j] * tau[j].x;
        acc.y += S0[6 * i + j] * tau[j].y;
      }
      o[i] = acc;
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) tau[c] = cscale(o[c], -s);
    return;
  }
  const float A00 = K[3] * K[5] - K[4] * K[4];
  const float A01 = K[2] * K[4] - K[1] * K[5];
  const float A02 = K[1] * K[4] - K[2] * K[3];
  const float A11 = K[0] * K[5] - K[2] * K[2];
  const float A12 = K[1] * K[2] - K[0] * K[4];
  const float A22 = K[0] * K[3] - K[1] * K[1];
  // K^{-1} = adj(K) / det: the adjugate here, 1/det folded into the scale
  const float rdet = fast_rcp(K[0] * A00 + K[1] * A01 + K[2] * A02);
  const float Nm[3][3] = {{A00, A01, A02}, {A01, A11, A12}, {A02, A12, A22}};
  // t = tau xi (tau symmetric, Voigt xx yy zz yz xz xy)
  float2 tv[3];
  tv[0] = make_float2(tau[0].x * xi[0] + tau[5].x * xi[1] + tau[4].x * xi[2],
                      tau[0].y * xi[0] + tau[5].y * xi[1] + tau[4].y * xi[2]);
  tv[1] = make_float2(tau[5].x * xi[0] + tau[1].x * xi[1] + tau[3].x * xi[2],
                      tau[5].y * xi[0] + tau[1].y * xi[1] + tau[3].y * xi[2]);
  tv[2] = make_float2(tau[4].x * xi[0] + tau[3].x * xi[1] + tau[2].x * xi[2],
                      tau[4].y * xi[0] + tau[3].y * xi[1] + tau[2].y * xi[2]);
  float2 u[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    u[i] = make_float2(Nm[i][0] * tv[0].x + Nm[i][1] * tv[1].x + Nm[i][2] * tv[2].x,
                       Nm[i][0] * tv[0].y + Nm[i][1] * tv[1].y + Nm[i][2] * tv[2].y);
  // eps = -sym(xi (x) u) / N
  const float g = -s * rdet, h = 0.5f * g;
  tau[0] = cscale(u[0], g * xi[0]);
  tau[1] = cscale(u[1], g * xi[1]);
  tau[2] = cscale(u[2], g * xi[2]);
  tau[3] = make_float2(h * (xi[1] * u[2].x + xi[2] * u[1].x), h * (xi[1] * u[2].y + xi[2] * u[1].y));
  tau[4] = make_float2(h * (xi[0] * u[2].x + xi[2] * u[0].x), h * (xi[0] * u[2].y + xi[2] * u[0].y));
  tau[5] = make_float2(h * (xi[0] * u[1].x + xi[1] * u[0].x), h * (xi[0] * u[1].y + xi[1] * u[0].y));
}

// Column tiles of a z pass per instance: C consecutive kx of one ky row, then,
// with a Nyquist plane, C consecutive ky of that plane (kx = nx/2).
__host__ __device__ inline int z_tiles_inst(const KArgs& a, int C) {
  const int rows = ((a.ncol + C - 1) / C) * a.ny;
  return a.nq_row ? rows : rows + (a.ny + C - 1) / C;
}

// The column of thread cc of logical block lb of a one-dimensional z-pass
// grid (z_tiles_inst blocks per instance).
struct ZCol {
  int inst, kx, ky;
  bool valid;
  bool first;    // the block holding xi = 0 of its instance (row tile 0 of ky 0)
  float2* col;   // element kz = 0 of component 0
  size_t zs;     // stride between consecutive kz
};

__device__ __forceinline__ ZCol z_col(const KArgs& a, int lb, int C, int cc) {
  const int ntile = (a.ncol + C - 1) / C;
  const int per = z_tiles_inst(a, C);
  ZCol z;
  z.inst = lb / per;
  const int r = lb % per;
  if (r < ntile * a.ny) {
    const int tile = r % ntile;
    z.ky = r / ntile;
    z.kx = tile * C + cc;
    z.valid = z.kx < a.ncol;
    z.first = r == 0;
    z.zs = (size_t)a.ny * a.sh;
    z.col = a.spec + (size_t)z.inst * a.nz * z.zs + (size_t)z.ky * a.sh + (z.valid ? z.kx : 0);
  } else {
    z.kx = a.nx / 2;
    z.ky = (r - ntile * a.ny) * C + cc;
    z.valid = z.ky < a.ny;
    z.first = false;
    z.zs = a.ny;
    z.col = a.spec + a.nqo + (size_t)z.inst * a.nz * a.ny + (z.valid ? z.ky : 0);
  }
  return z;
}

// The same for a three-dimensional z-pass grid: x the row tiles, then (with a
// Nyquist plane) one more index whose blocks take the plane's tiles; y the
// row ky of an instance (ky + instance ny), or the plane tile (ky < its count;
// the other blocks of that x index hold no column).
__host__ __device__ inline int z_tiles_x(const KArgs& a, int C) {
  return (a.ncol + C - 1) / C + (a.nq_row ? 0 : 1);
}

__device__ __forceinline__ ZCol z_col3(const KArgs& a, int bx, int by, int C, int cc) {
  const int ntile = (a.ncol + C - 1) / C;
  ZCol z;
  z.inst = by / a.ny;
  const int r = by % a.ny;
  if (bx < ntile) {
    z.ky = r;
    z.kx = bx * C + cc;
    z.valid = z.kx < a.ncol;
    z.first = bx == 0 && r == 0;
    z.zs = (size_t)a.ny * a.sh;
    z.col = a.spec + (size_t)z.inst * a.nz * z.zs + (size_t)z.ky * a.sh + (z.valid ? z.kx : 0);
  } else {
    z.kx = a.nx / 2;
    z.ky = r * C + cc;
    z.valid = z.ky < a.ny;
    z.first = false;
    z.zs = a.ny;
    z.col = a.spec + a.nqo + (size_t)z.inst * a.nz * a.ny + (z.valid ? z.ky : 0);
  }
  return z;
}

__device__ inline void fin_ms(const KArgs& a, int inst, int nblk, double* scratch, double* ebar_out);

// z pass of the fixed point: forward z transform of the six polarisation
// components, Green's operator, inverse z transform. 1D grid of
// (column tile, ky) blocks in XCD-aware order; tiles of kZmsTile columns.
// The block holding xi = 0 of an instance first applies the mixed condition
// (the mean strain of the next iterate from the stress sums of the forward
// x pass, nblk_x blocks), so no separate launch sits between the passes.
template <int N, int C, int PK>
__global__ __launch_bounds__((col_threads<N, PK, C>())) void k_z_ms(const KArgs a, int nblk_x) {
  using P = PV<N, PK>;
  constexpr int E = P::E, T = N / E;
  // two pencils per LDS exchange round (half the barriers of one at a time)
  // where their two buffers fit in 64 KiB
  constexpr int NC = (2 * N * C * 8 <= 65536) ? 2 : 1;
  __shared__ float2 lds[NC * N * C];
  __shared__ double ebar[6];
  const int cc = threadIdx.x % C, t = threadIdx.x / C;
  const ZCol zc = z_col(a, xcd_logical(blockIdx.x, gridDim.x), C, cc);
  const int inst = zc.inst, kx = zc.kx, ky = zc.ky;
  const bool valid = zc.valid;
  const DevState* st = a.state + inst;
  if (st->st.done) return;
  if (zc.first) {
    // the pass's LDS (NC N C float2 >= blockDim doubles) is free until the transforms
    fin_ms(a, inst, nblk_x, reinterpret_cast<double*>(lds), ebar);
    __syncthreads();
  }
  const ctab_t ref = (ctab_t)(a.ref + (size_t)inst * kRefStride);
  const size_t cs = a.cs;
  const size_t zs = zc.zs;
  float2* col = zc.col;
  float2 v[6][E];
#pragma unroll
  for (int c = 0; c < 6; ++c)
#pragma unroll
    for (int m = 0; m < E; ++m)
      v[c][m] = valid ? col[c * cs + (size_t)(t + T * m) * zs] : make_float2(0.f, 0.f);
  TwCache<N, P, 1> twf;
  twf.load(a.tw_z, t);
  ColView<C> views[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) views[c] = ColView<C>{lds + c * N * C + cc};
#pragma unroll
  for (int g = 0; g < 6; g += NC)
    fft_pencils<N, 1, P, NC>(*reinterpret_cast<float2(*)[NC][E]>(&v[g]), views, t, twf);
  const int kxv = valid ? kx : 0;
  float xi[3] = {(float)kxv / (float)a.nx, (float)signed_k(ky, a.ny) / (float)a.ny, 0.f};
  const float inz = 1.f / (float)a.nz;
  float K0[6], K1[6], K2[6];
  acoustic_parts(ref, xi[0], xi[1], K0, K1, K2);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int kz = t + T * m;
    xi[2] = (float)signed_k(kz, a.nz) * inz;
    float K[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) K[e] = K0[e] + xi[2] * (K1[e] + xi[2] * K2[e]);
    float2 tau[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) tau[c] = v[c][m];
    green_apply(a, ebar, ref + 21, kxv, ky, kz, xi, K, tau);
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c][m] = tau[c];
  }
  const TwCache<N, P, -1> twi = twf.conj();
#pragma unroll
  for (int g = 0; g < 6; g += NC)
    fft_pencils<N, -1, P, NC>(*reinterpret_cast<float2(*)[NC][E]>(&v[g]), views, t, twi);
  // streaming stores (the loads stay plain: see gld)
  if (valid) {
#pragma unroll
    for (int c = 0; c < 6; ++c)
#pragma unroll
      for (int m = 0; m < E; ++m) gst(col + c * cs + (size_t)(t + T * m) * zs, v[c][m]);
  }
}

// z pass of the phase-field update for variant blockIdx.z: forward z
// transform, semi-implicit divide by 1 + 2 L dt kappa |xi|^2 (and 1/N),
// Parseval sum of |xi|^2 |f_hat|^2 of the new state, inverse transform.
// mode 1: Parseval sum of the unmodified spectrum only, nothing stored.
// WG: the gradient force may be wanted (a mobility field, or mode 2); without
// it the kernel holds one pencil less.
template <int N, bool GK, bool WG, int K>
__global__ __launch_bounds__((col_threads<N, K, kColTile>())) void k_z_ac(const KArgs a, int mode) {
  using P = PV<N, K>;
  constexpr int E = P::E, T = N / E, C = kColTile;
  __shared__ float2 lds[N * C];
  if (a.guard_ready && !a.state[0].st.ready) return;
  const int cc = threadIdx.x % C, t = threadIdx.x / C;
  const ZCol zc = z_col3(a, blockIdx.x, blockIdx.y, C, cc);
  const int kx = zc.kx, ky = zc.ky, inst = zc.inst, q = blockIdx.z;
  const bool valid = zc.valid;
  const size_t cs = a.cs;
  const size_t zs = zc.zs;
  // partials ordered [inst][variant][ky row][x index] so each instance's are contiguous
  const size_t blk = (((size_t)inst * a.nv + q) * a.ny + blockIdx.y % a.ny) * gridDim.x + blockIdx.x;
  if ((int)blockIdx.x >= (a.ncol + C - 1) / C && (int)(blockIdx.y % a.ny) * C >= a.ny) {
    // a plane index with no column: its partials are zero
    double en[kQgd] = {0.0, 0.0, 0.0};
    block_sum<kQgd>(en, a.part_gd + blk * kQgd);
    return;
  }
  float2* col = zc.col + q * cs;
  float2 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = valid ? gld(col + (size_t)(t + T * m) * zs) : make_float2(0.f, 0.f);
  TwCache<N, P, 1> twf;
  twf.load(a.tw_z, t);
  const ColView<C> view{lds + cc};
  fft_pencil<N, 1, P>(v, view, t, twf);
  const int sy = signed_k(ky, a.ny);
  const double wgt = (kx == 0 || kx == a.nx / 2) ? 1.0 : 2.0;
  const GradSym<GK> gs(a, inst, q, kx, sy);
  // the gradient force G = 2 div(K grad f) = -gscale sym f_hat of the new
  // state (with a mobility field) or of the given one (mode 2)
  const bool want_g = WG && (mode == 2 || (mode == 0 && a.lapf != nullptr));
  float2 g[E];
  float e0 = 0.f;  // this thread's Parseval terms, then FP64
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int sz = signed_k(t + T * m, a.nz);
    const float fz = (float)sz * (float)sz, cz = cross_k(sz, a.nz);
    if (mode == 0) v[m] = cscale(v[m], fast_rcp(gs.den(cz, fz)));
    const float sym = gs.sym(cz, fz);
    e0 += sym * (v[m].x * v[m].x + v[m].y * v[m].y);
    v[m] = cscale(v[m], a.inv_ntot);
    g[m] = want_g ? cscale(v[m], -a.gscale * sym) : make_float2(0.f, 0.f);
  }
  double en[kQgd] = {valid ? wgt * (double)e0 : 0.0, 0.0, 0.0};
  if (mode == 0) {
    fft_pencil<N, -1, P>(v, view, t, twf.conj());
    if (valid) {
#pragma unroll
      for (int m = 0; m < E; ++m) gst(col + (size_t)(t + T * m) * zs, v[m]);
    }
  }
  if (want_g) {
    fft_pencil<N, -1, P>(g, view, t, twf.conj());
    float2* gcol = mode == 2 ? col : col + (size_t)a.nv * cs;
    if (valid) {
#pragma unroll
      for (int m = 0; m < E; ++m) gst(gcol + (size_t)(t + T * m) * zs, g[m]);
    }
  }
  block_sum<kQgd>(en, a.part_gd + blk * kQgd);
}

// Plain z transform (checking the passes) with the Allen-Cahn z pass's plan.
template <int N, int DIR, int K>
__global__ __launch_bounds__((col_threads<N, K, kColTile>())) void k_z_raw(const KArgs a) {
  using P = PV<N, K>;
  constexpr int E = P::E, T = N / E, C = kColTile;
  __shared__ float2 lds[N * C];
  const int cc = threadIdx.x % C, t = threadIdx.x / C;
  if ((int)blockIdx.x >= (a.ncol + C - 1) / C && (int)(blockIdx.y % a.ny) * C >= a.ny) return;  // no column
  const ZCol zc = z_col3(a, blockIdx.x, blockIdx.y, C, cc);
  const bool valid = zc.valid;
  const size_t zs = zc.zs;
  float2* col = zc.col + blockIdx.z * a.cs;
  float2 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = valid ? col[(size_t)(t + T * m) * zs] : make_float2(0.f, 0.f);
  TwCache<N, P, DIR> tw;
  tw.load(a.tw_z, t);
  fft_pencil<N, DIR, P>(v, ColView<C>{lds + cc}, t, tw);
  if (valid) {
#pragma unroll
    for (int m = 0; m < E; ++m) col[(size_t)(t + T * m) * zs] = v[m];
  }
}

// ------------------------------------------------- per-grain gradient tensors
// With per-grain tensors K_a^g the implicit step takes kbar_a I (the largest
// eigenvalue over the grains) and the remainder 2 div((K_a(x) - kbar_a I)
// grad f_a) enters the update explicitly at f^n. It is formed with spectral
// first derivatives i xi_j (xi_j zero at a Nyquist index, where the
// derivative, odd in it, has no value), in three passes around raw x and y
// transforms: gradient (z), flux (x), divergence (z).

// First-derivative wave numbers of a column (kx, ky) of a z pass.
__device__ __forceinline__ void deriv_xy(const KArgs& a, int kx, int ky, float& dxk, float& dyk) {
  dxk = kx == a.nx / 2 ? 0.f : a.cdx * (float)kx;
  const int sy = signed_k(ky, a.ny);
  dyk = 2 * sy == -a.ny ? 0.f : a.cdy * (float)sy;
}

__device__ __forceinline__ float deriv_z(const KArgs& a, int kz) {
  const int sz = signed_k(kz, a.nz);
  return 2 * sz == -a.nz ? 0.f : a.cdz * (float)sz;
}

// Gradient: the (x, y)-transformed f_q (components 0..V-1) -> forward z
// transform, i xi_j f_hat for j = x, y, z, inverse z transforms into
// components 3q + j. Variants are taken from the last down, so each output
// component is written after the input it replaces has been read.
template <int N, int K>
__global__ __launch_bounds__((col_threads<N, K, kColTile>())) void k_z_grad(const KArgs a) {
  using P = PV<N, K>;
  constexpr int E = P::E, T = N / E, C = kColTile;
  __shared__ float2 lds[N * C];
  if (a.guard_ready && !a.state[0].st.ready) return;
  const int cc = threadIdx.x % C, t = threadIdx.x / C;
  if ((int)blockIdx.x >= (a.ncol + C - 1) / C && (int)(blockIdx.y % a.ny) * C >= a.ny) return;  // no column
  const ZCol zc = z_col3(a, blockIdx.x, blockIdx.y, C, cc);
  const bool valid = zc.valid;
  const size_t zs = zc.zs;
  float dk[3];
  deriv_xy(a, zc.kx, zc.ky, dk[0], dk[1]);
  TwCache<N, P, 1> twf;
  twf.load(a.tw_z, t);
  const TwCache<N, P, -1> twi = twf.conj();
  const ColView<C> view{lds + cc};
#pragma unroll 1
  for (int q = a.nv - 1; q >= 0; --q) {
    const float2* in = zc.col + q * a.cs;
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = valid ? in[(size_t)(t + T * m) * zs] : make_float2(0.f, 0.f);
    fft_pencil<N, 1, P>(v, view, t, twf);
#pragma unroll 1
    for (int j = 0; j < 3; ++j) {
      float2 w[E];
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const float xi = j < 2 ? dk[j] : deriv_z(a, t + T * m);
        w[m] = make_float2(-xi * v[m].y, xi * v[m].x);
      }
      fft_pencil<N, -1, P>(w, view, t, twi);
      float2* out = zc.col + (3 * q + j) * a.cs;
      if (valid) {
#pragma unroll
        for (int m = 0; m < E; ++m) out[(size_t)(t + T * m) * zs] = w[m];
      }
    }
  }
}

// Divergence into the update: the (x, y)-transformed flux components, held
// from component V on (V + 3q + j), -> forward z transforms, 2 sum_j i xi_j
// q_hat_j, inverse z transform, added times L dt / nz (the z transforms carry
// nz) to component q: the update's right-hand side f - L dt (chem - mech)
// after its x and y transforms, so the update gains + L dt 2 div((K - kbar I)
// grad f^n) before its z pass.
template <int N, int K>
__global__ __launch_bounds__((col_threads<N, K, kColTile>())) void k_z_div(const KArgs a) {
  using P = PV<N, K>;
  constexpr int E = P::E, T = N / E, C = kColTile;
  __shared__ float2 lds[N * C];
  if (a.guard_ready && !a.state[0].st.ready) return;
  const int cc = threadIdx.x % C, t = threadIdx.x / C;
  if ((int)blockIdx.x >= (a.ncol + C - 1) / C && (int)(blockIdx.y % a.ny) * C >= a.ny) return;  // no column
  const ZCol zc = z_col3(a, blockIdx.x, blockIdx.y, C, cc);
  const bool valid = zc.valid;
  const size_t zs = zc.zs;
  float dk[3];
  deriv_xy(a, zc.kx, zc.ky, dk[0], dk[1]);
  TwCache<N, P, 1> twf;
  twf.load(a.tw_z, t);
  const TwCache<N, P, -1> twi = twf.conj();
  const ColView<C> view{lds + cc};
  const float w = a.LDt / (float)a.nz;
#pragma unroll 1
  for (int q = 0; q < a.nv; ++q) {
    float2 acc[E];
#pragma unroll
    for (int m = 0; m < E; ++m) acc[m] = make_float2(0.f, 0.f);
#pragma unroll 1
    for (int j = 0; j < 3; ++j) {
      const float2* in = zc.col + (a.nv + 3 * q + j) * a.cs;
      float2 v[E];
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = valid ? in[(size_t)(t + T * m) * zs] : make_float2(0.f, 0.f);
      fft_pencil<N, 1, P>(v, view, t, twf);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const float xi = 2.f * (j < 2 ? dk[j] : deriv_z(a, t + T * m));
        acc[m].x -= xi * v[m].y;
        acc[m].y += xi * v[m].x;
      }
    }
    fft_pencil<N, -1, P>(acc, view, t, twi);
    float2* out = zc.col + q * a.cs;
    if (valid) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        float2* o = out + (size_t)(t + T * m) * zs;
        const float2 r = *o;
        *o = make_float2(r.x + w * acc[m].x, r.y + w * acc[m].y);
      }
    }
  }
}

// Flux, x pass: per row and variant q, the inverse x transforms of the three
// gradient components (scaled by 1/N: grad f), the flux (K_q^g - kbar_q I)
// grad f with g the voxel's grain, the sum of grad f . flux (FP64 per block:
// the remainder's gradient energy), and the forward x transforms of the flux
// into the same components.
template <int M>
__global__ __launch_bounds__(xthreads<M>()) void k_x_flux(const KArgs a) {
  constexpr int E = XPlan<M>::E, T = M / E, ROWS = xthreads<M>() / T;
  constexpr int LROW = RowView::padded(M) + 1;
  __shared__ float2 lds[ROWS * LROW];
  if (a.guard_ready && !a.state[0].st.ready) return;
  const int t = threadIdx.x % T, p = threadIdx.x / T;
  const int nrows = a.ninst * a.nz * a.ny;
  const int row = blockIdx.x * ROWS + p;
  const bool valid = row < nrows;
  const size_t rowv = valid ? row : 0;
  const size_t rbase = rowv * a.nx;
  const float s = a.inv_ntot;
  XTw<M, -1> twi;
  twi.load(a, t);
  XTw<M, 1> twf;
  twf.load(a, t);
  float en = 0.f;
#pragma unroll 1
  for (int q = 0; q < a.nv; ++q) {
    float2 g[3][E];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      c2r_row<M>(g[j], lds + p * LROW, t, valid, a.spec + (3 * q + j) * a.cs + rowv * a.sh,
                 nyq_at(a, 3 * q + j, rowv), twi);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const size_t x0 = rbase + 2 * (t + T * m);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int gr = a.gid ? a.gid[x0 + h] : 0;
        const float* kr = a.krem + ((size_t)gr * a.nv + q) * 6;
        const float gx = s * (h ? g[0][m].y : g[0][m].x);
        const float gy = s * (h ? g[1][m].y : g[1][m].x);
        const float gz = s * (h ? g[2][m].y : g[2][m].x);
        const float fx = kr[0] * gx + kr[5] * gy + kr[4] * gz;
        const float fy = kr[5] * gx + kr[1] * gy + kr[3] * gz;
        const float fz = kr[4] * gx + kr[3] * gy + kr[2] * gz;
        if (valid) en += gx * fx + gy * fy + gz * fz;
        if (h) {
          g[0][m].y = fx; g[1][m].y = fy; g[2][m].y = fz;
        } else {
          g[0][m].x = fx; g[1][m].x = fy; g[2][m].x = fz;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 3; ++j)
      r2c_one<M>(g[j], lds + p * LROW, t, valid, a.spec + (3 * q + j) * a.cs + rowv * a.sh,
                 nyq_at(a, 3 * q + j, rowv), twf);
  }
  double acc[1] = {(double)en};
  block_sum<1, xthreads<M>() / 64>(acc, a.part_rem + blockIdx.x);
}

// z pass of the homogeneous spectral path (one stiffness C per instance,
// linear h, no plastic strain) for V variants. With a single stiffness the
// equilibrium stress is known in closed form per wavevector, so no fixed
// point is needed: for xi != 0,
//   sigma_hat : eps0_a = -sum_b B_ab(n) f_hat_b,
//   B_ab(n) = eps0_a : C : eps0_b - (sigma0_a n) . K(n)^{-1} (sigma0_b n),
// with sigma0_a = C : eps0_a and K(n) = C n n; B = 0 at the ambiguous Nyquist
// wavevectors (stress-free there, as in the fixed point). At xi = 0 the mean
// strain follows from the mixed condition (kh_begin_mean). Components 0..V-1 hold f_hat on
// entry and the new order parameters' spectra on exit; V..2V-1 hold the
// transform of f - L dt chem. FP64 partials: gradient sum of the new state
// and the fluctuation part of the elastic energy.
template <int V>
__host__ __device__ constexpr int kh_tile() { return V == 1 ? kColTile : kZmsTile; }
// the tile the spectral z pass runs with: the group's tuned one, else the default
__host__ __device__ inline int kh_tile_of(const KArgs& a) {
  return a.ztile_kh ? a.ztile_kh : (a.nv == 1 ? kColTile : kZmsTile);
}

// mode 1: instead of the update, L dt dF/df of the state whose transforms
// are in components 0..V-1 (f_hat) and V..2V-1 (L dt chem_hat):
// L dt (chem_hat + 2 kappa |xi|^2 f_hat - mech_hat); no energy sums.
// mode 2: the same with the gradient term taken on components 2V..3V-1
// (w_hat) instead of f_hat: L dt (chem_hat + 2 kappa |xi|^2 w_hat -
// mech_hat(f_hat)), the macro-step residual's force (k_x_fwd_ct).
__device__ inline void kh_begin_mean(const KArgs& a, int inst, int nblk, double* scratch);

template <int N, int V, bool GK, int C, int PK>
__global__ __launch_bounds__((col_threads<N, PK, C>())) void k_z_kh(const KArgs a, int mode, int nblk_x) {
  using P = PV<N, PK>;
  constexpr int E = P::E, T = N / E;
  __shared__ float2 lds[N * C];
  const int cc = threadIdx.x % C, t = threadIdx.x / C;
  const int lb = xcd_logical(blockIdx.x, gridDim.x);
  const ZCol zc = z_col(a, lb, C, cc);
  const int kx = zc.kx, ky = zc.ky, inst = zc.inst;
  const bool valid = zc.valid;
  if (zc.first) {
    // this block holds xi = 0: the mean fields of the instance first
    // the pass's LDS (N C float2 >= blockDim doubles) is free until the transforms
    kh_begin_mean(a, inst, nblk_x, reinterpret_cast<double*>(lds));
    __syncthreads();
  }
  const ctab_t kt = (ctab_t)(a.kh + (size_t)inst * kKhStride);
  const size_t cs = a.cs;
  const size_t zs = zc.zs;
  float2* col = zc.col;
  float2 th[V][E], rh[V][E];
#pragma unroll
  for (int q = 0; q < V; ++q)
#pragma unroll
    for (int m = 0; m < E; ++m) {
      th[q][m] = valid ? col[q * cs + (size_t)(t + T * m) * zs] : make_float2(0.f, 0.f);
      rh[q][m] = valid ? col[(V + q) * cs + (size_t)(t + T * m) * zs] : make_float2(0.f, 0.f);
    }
  TwCache<N, P, 1> twf;
  twf.load(a.tw_z, t);
  const ColView<C> view{lds + cc};
#pragma unroll
  for (int q = 0; q < V; ++q) {
    fft_pencil<N, 1, P>(th[q], view, t, twf);
    fft_pencil<N, 1, P>(rh[q], view, t, twf);
  }
  const int kxv = valid ? kx : 0;
  const int sy = signed_k(ky, a.ny);
  const float xi0 = (float)kxv / (float)a.nx, xi1 = (float)sy / (float)a.ny;
  float K0[6], K1[6], K2[6];
  acoustic_parts(kt, xi0, xi1, K0, K1, K2);
  // sigma0_a xi = u0_a + xi_z u1_a
  float u0[V][3], u1[V][3];
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const ctab_t s0 = kt + 21 + 6 * q;
    u0[q][0] = s0[0] * xi0 + s0[5] * xi1;
    u0[q][1] = s0[5] * xi0 + s0[1] * xi1;
    u0[q][2] = s0[4] * xi0 + s0[3] * xi1;
    u1[q][0] = s0[4];
    u1[q][1] = s0[3];
    u1[q][2] = s0[2];
  }
  const ctab_t W = kt + 21 + 6 * kMaxVar;
  const float fx = (float)kxv * (float)kxv, fy = (float)sy * (float)sy;
  const double wgt = (kxv == 0 || kxv == a.nx / 2) ? 1.0 : 2.0;
  const float inz = 1.f / (float)a.nz;
  GradSym<GK> gsq[V];
#pragma unroll
  for (int q = 0; q < V; ++q) gsq[q] = GradSym<GK>(a, inst, q, kxv, sy);
  if (mode == 2) {
    // gradient force of w into the chemical part, one variant at a time
#pragma unroll
    for (int q = 0; q < V; ++q) {
      float2 w[E];
#pragma unroll
      for (int m = 0; m < E; ++m)
        w[m] = valid ? col[(2 * V + q) * cs + (size_t)(t + T * m) * zs] : make_float2(0.f, 0.f);
      fft_pencil<N, 1, P>(w, view, t, twf);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int sz = signed_k(t + T * m, a.nz);
        const float g = gsq[q].den(cross_k(sz, a.nz), (float)sz * (float)sz) - 1.f;
        rh[q][m].x += g * w[m].x;
        rh[q][m].y += g * w[m].y;
      }
    }
  }
  float ef[kQgd] = {0.f, 0.f, 0.f};  // this thread's terms, then FP64
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int kz = t + T * m;
    const int sz = signed_k(kz, a.nz);
    const float xi2 = (float)sz * inz;
    const float fz = (float)sz * (float)sz;
    float2 y[V];  // sum_b B_ab f_hat_b
#pragma unroll
    for (int q = 0; q < V; ++q) y[q] = make_float2(0.f, 0.f);
    const bool dc = kxv == 0 && ky == 0 && kz == 0;
    if (!dc && !ambiguous_nyquist(a, kxv, ky, kz)) {
      float K[6];
#pragma unroll
      for (int e = 0; e < 6; ++e) K[e] = K0[e] + xi2 * (K1[e] + xi2 * K2[e]);
      const float A00 = K[3] * K[5] - K[4] * K[4];
      const float A01 = K[2] * K[4] - K[1] * K[5];
      const float A02 = K[1] * K[4] - K[2] * K[3];
      const float A11 = K[0] * K[5] - K[2] * K[2];
      const float A12 = K[1] * K[2] - K[0] * K[4];
      const float A22 = K[0] * K[3] - K[1] * K[1];
      const float rdet = fast_rcp(K[0] * A00 + K[1] * A01 + K[2] * A02);
      float u[V][3], nu[V][3];
#pragma unroll
      for (int q = 0; q < V; ++q) {
#pragma unroll
        for (int i = 0; i < 3; ++i) u[q][i] = u0[q][i] + xi2 * u1[q][i];
        nu[q][0] = (A00 * u[q][0] + A01 * u[q][1] + A02 * u[q][2]) * rdet;
        nu[q][1] = (A01 * u[q][0] + A11 * u[q][1] + A12 * u[q][2]) * rdet;
        nu[q][2] = (A02 * u[q][0] + A12 * u[q][1] + A22 * u[q][2]) * rdet;
      }
#pragma unroll
      for (int q = 0; q < V; ++q)
#pragma unroll
        for (int r = 0; r < V; ++r) {
          const float b = W[V * q + r] - (u[q][0] * nu[r][0] + u[q][1] * nu[r][1] + u[q][2] * nu[r][2]);
          y[q].x += b * th[r][m].x;
          y[q].y += b * th[r][m].y;
        }
      if (mode == 0) {
#pragma unroll
        for (int q = 0; q < V; ++q) ef[1] += th[q][m].x * y[q].x + th[q][m].y * y[q].y;
      }
    }
    const float cz = cross_k(sz, a.nz);
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const float den = gsq[q].den(cz, fz);
      const float rden = fast_rcp(den);
      const float x2 = gsq[q].sym(cz, fz);
      if (mode == 0) ef[2] += x2 * (th[q][m].x * th[q][m].x + th[q][m].y * th[q][m].y);
      float2 nv;
      if (mode == 0) {
        nv = make_float2((rh[q][m].x - a.LDt * y[q].x) * rden, (rh[q][m].y - a.LDt * y[q].y) * rden);
        if (dc && valid) nv = make_float2(rh[q][m].x + (float)a.state[inst].kh_drive[q], 0.f);
        ef[0] += x2 * (nv.x * nv.x + nv.y * nv.y);
      } else {
        // mode 2: the gradient term is already in rh
        const float g = mode == 1 ? den - 1.f : 0.f;
        nv = make_float2(rh[q][m].x + g * th[q][m].x + a.LDt * y[q].x, rh[q][m].y + g * th[q][m].y + a.LDt * y[q].y);
        if (dc && valid) nv = make_float2(rh[q][m].x - (float)a.state[inst].kh_drive[q], 0.f);
      }
      th[q][m] = cscale(nv, a.inv_ntot);
    }
  }
  const TwCache<N, P, -1> twi = twf.conj();
#pragma unroll
  for (int q = 0; q < V; ++q) fft_pencil<N, -1, P>(th[q], view, t, twi);
  if (valid) {
#pragma unroll
    for (int q = 0; q < V; ++q)
#pragma unroll
      for (int m = 0; m < E; ++m) col[q * cs + (size_t)(t + T * m) * zs] = th[q][m];
  }
  if (mode == 0) {
    double en[kQgd];
#pragma unroll
    for (int q = 0; q < kQgd; ++q) en[q] = valid ? wgt * (double)ef[q] : 0.0;
    block_sum<kQgd>(en, a.part_gd + (size_t)lb * kQgd);
  }
}

// Residual of a macro step, inverse x pass: r = f~ - prev + S g with g the
// inverse transform of components 0..V-1 (L dt dF/df); per-block max |r|.
template <int M>
__global__ __launch_bounds__(xthreads<M>()) void k_x_resid(const KArgs a, const float* __restrict__ prev,
                                                          float S) {
  constexpr int E = XPlan<M>::E, T = M / E, ROWS = xthreads<M>() / T;
  constexpr int LROW = RowView::padded(M) + 1;
  __shared__ float2 lds[ROWS * LROW];
  const int t = threadIdx.x % T, p = threadIdx.x / T;
  const int nrows = a.ninst * a.nz * a.ny;
  const int row = blockIdx.x * ROWS + p;
  const bool valid = row < nrows;
  const size_t vs = (size_t)nrows * a.nx;
  const size_t rbase = (size_t)(valid ? row : 0) * a.nx;
  const size_t cs = a.cs;
  float mx = 0.f;
  XTw<M, -1> tw;
  tw.load(a, t);
#pragma unroll 1
  for (int q = 0; q < a.nv; ++q) {
    float2 v[E];
    c2r_row<M>(v, lds + p * LROW, t, valid, a.spec + q * cs + (size_t)(valid ? row : 0) * a.sh,
               nyq_at(a, q, valid ? row : 0), tw);
    if (valid) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const size_t off = q * vs + rbase + 2 * (t + T * m);
        const float2 f = *reinterpret_cast<const float2*>(a.eta + off);
        const float2 f0 = *reinterpret_cast<const float2*>(prev + off);
        const float r0 = f.x - f0.x + S * v[m].x, r1 = f.y - f0.y + S * v[m].y;
        // NaN propagates through fmaxf only if both are NaN: count it as huge
        mx = fmaxf(mx, isfinite(r0) ? fabsf(r0) : 3.0e38f);
        mx = fmaxf(mx, isfinite(r1) ? fabsf(r1) : 3.0e38f);
      }
    }
    __syncthreads();
  }
  block_minmax(0.f, mx, a.part_mm + 2 * (size_t)blockIdx.x);
}


// ------------------------------------------------------------ small kernels
// One thread per instance: take the step's load, reset the iteration status,
// shift the history of converged mean strains (the field in memory is the
// latest converged one) and set the mean of the first iterate: the load for
// strain-controlled components, the extrapolated mean (as the field itself)
// for stress-controlled ones.
__global__ void k_step_begin(const KArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.ninst) return;
  DevState* st = a.state + i;
  const double* ld = a.loads + 12 * (size_t)i;
  for (int c = 0; c < 6; ++c) {
    st->ebar_h[3][c] = st->ebar_h[2][c];
    st->ebar_h[2][c] = st->ebar_h[1][c];
    st->ebar_h[1][c] = st->ebar_h[0][c];
    st->ebar_h[0][c] = st->ebar_field[c];
    const double l = st->ebar_h[0][c], p1 = st->ebar_h[1][c], p2 = st->ebar_h[2][c], p3 = st->ebar_h[3][c];
    const double base = a.iter_mode == 3   ? 4.0 * (l + p2) - 6.0 * p1 - p3
                        : a.iter_mode == 2 ? 3.0 * (l - p1) + p2
                        : a.iter_mode == 1 ? 2.0 * l - p1
                                           : l;
    st->ebar_base[c] = base;
    st->eps_target[c] = ld[c];
    st->sig_target[c] = ld[6 + c];
    st->ebar_cur[c] = ((a.stress_mask >> c) & 1u) ? base : ld[c];
  }
  st->st.done = 0;
  st->st.iters = 0;
}

// state[0].st.ready = every instance of the group has converged (one block);
// the update passes of a step replayed as a graph run only then.
__global__ __launch_bounds__(256) void k_group_ready(const KArgs a) {
  __shared__ int all;
  if (threadIdx.x == 0) all = 1;
  __syncthreads();
  for (int i = threadIdx.x; i < a.ninst; i += blockDim.x)
    if (!a.state[i].st.done) all = 0;
  __syncthreads();
  if (threadIdx.x == 0) a.state[0].st.ready = all;
}

// Mean of each strain component of instance j of a caller-set field (one
// block per component, FP64, fixed summation order): the mean strain the
// field in memory carries, taken as the base of the next step's first
// iterate.
__global__ __launch_bounds__(1024) void k_strain_mean(const KArgs a, const float* __restrict__ f, int j) {
  __shared__ double part[1024];
  const int c = blockIdx.x;
  const size_t nvox = (size_t)a.nx * a.ny * a.nz;
  const float* src = f + ((size_t)c * a.ninst + j) * nvox;
  double acc = 0.0;
  for (size_t i = threadIdx.x; i < nvox; i += blockDim.x) acc += (double)src[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h /= 2) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.state[j].ebar_field[c] = part[0] / (double)nvox;
}

// -------------------------------------------------------------- finalizes
// Deterministic sum over nblk blocks of Q partials ([nblk][Q], FP64). The
// block reads the array as one flat run with a stride S that is a multiple
// of Q, so a thread always meets the same quantity (q = thread mod Q) and
// every load is coalesced; sixteen loads are in flight per thread. The
// per-thread sums of a quantity are then added by a fixed pairwise tree in
// LDS. scratch: blockDim.x doubles of LDS.
template <int Q>
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int nblk, double (&out)[Q],
                                             double* scratch) {
  __shared__ double res[Q];
  const int t = threadIdx.x;
  const int S = (int)(blockDim.x / Q) * Q;
  const int total = nblk * Q;
  double acc = 0.0;
  if (t < S) {
    int i = t;
    for (; i + 15 * S < total; i += 16 * S) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = part[i + u * S];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc += v[u];
    }
    for (; i < total; i += S) acc += part[i];
  }
  scratch[t] = acc;
  __syncthreads();
  // entry t holds quantity t % Q, term j = t / Q of S / Q
  const int nt = S / Q, j = t / Q;
  for (int h = 1; h < nt; h *= 2) {
    if (t < S && j % (2 * h) == 0 && j + h < nt) scratch[t] += scratch[t + h * Q];
    __syncthreads();
  }
  if (t < Q) res[t] = scratch[t];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q) out[q] = res[q];
  __syncthreads();
}

// Partial-sum blocks per instance written by the z passes: the Allen-Cahn
// pass (16-column tiles, one per variant), the spectral path (16 columns for
// one variant, else 8).
__host__ __device__ inline int z_partials_inst(const KArgs& a, int mode) {
  if (mode == 2) return z_tiles_inst(a, kh_tile_of(a));
  return z_tiles_x(a, kColTile) * a.ny * a.nv;
}

// Mixed condition after the forward x pass of an iteration: the mean strain
// of the next iterate, into the state and into ebar_out (LDS of the caller).
__device__ inline void fin_ms(const KArgs& a, int inst, int nblk, double* scratch, double* ebar_out) {
  DevState* st = a.state + inst;
  double s[kQms];
  sum_partials<kQms>(a.part_ms + (size_t)inst * nblk * kQms, nblk, s, scratch);
  if (threadIdx.x != 0) return;
  const double* Bss = a.bss + 36 * (size_t)inst;
  const double ntot = (double)a.nx * a.ny * a.nz;
  double r[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) r[c] = s[c] / ntot - st->sig_target[c];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double e;
    if ((a.stress_mask >> i) & 1u) {
      double d = 0.0;
#pragma unroll
      for (int j = 0; j < 6; ++j)
        if ((a.stress_mask >> j) & 1u) d += Bss[6 * i + j] * r[j];
      e = st->ebar_cur[i] - d;
    } else {
      e = st->eps_target[i];
    }
    st->ebar_next[i] = e;
    ebar_out[i] = e;
  }
}

// Convergence test after the inverse x pass of an iteration.
__device__ inline void fin_res(const KArgs& a, int inst, int nblk, double* scratch) {
  DevState* st = a.state + inst;
  double s[kQres];
  sum_partials<kQres>(a.part_res + (size_t)inst * nblk * kQres, nblk, s, scratch);
  if (threadIdx.x != 0) return;
  const double r = s[1] > 0.0 ? sqrt(s[0] / s[1]) : (s[0] > 0.0 ? 1.0e300 : 0.0);
  st->st.residual = r;
  st->st.iters += 1;
  st->st.done = r <= a.tol ? 1 : 0;
  // a non-finite strain never converges: stop iterating and report it
  if (!isfinite(s[0]) || !isfinite(s[1])) {
    st->st.nonfinite = 1;
    st->st.done = 1;
  }
  for (int c = 0; c < 6; ++c) {
    st->ebar_field[c] = st->ebar_next[c];
    st->ebar_cur[c] = st->ebar_next[c];
    st->ebar_base[c] = st->ebar_next[c];
  }
}

// Stats of the step (raw sums; the host scales them) and the gradient sum of
// the new state. mode 0: fixed-point path; 1: only the gradient sum of the
// initial state; 2: homogeneous spectral path (stress, strain and the
// mean-field elastic energy from the mean kernel).
// The four reductions run in four blocks of one launch (part 0: gradient
// sums, 1: energies and means, 2: non-finite count, 3: extrema); each writes
// its own fields of the state.
__device__ inline void fin_ac(const KArgs& a, int inst, int nblk_x, int nblk_z, int mode, int part,
                              double* scratch) {
  DevState* st = a.state + inst;
  if (part == 0) {
    double gd[kQgd];
    sum_partials<kQgd>(a.part_gd + (size_t)inst * nblk_z * kQgd, nblk_z, gd, scratch);
    // per-grain tensors: the remainder's energy of the starting state, from this step's flux pass
    double rem[1] = {0.0};
    if (a.part_rem && mode == 0) sum_partials<1>(a.part_rem + (size_t)inst * nblk_x, nblk_x, rem, scratch);
    if (threadIdx.x != 0) return;
    if (mode == 1) {
      st->gd_cur = gd[0];
      return;
    }
    // the starting state's (the Parseval sums carry a factor N the host removes)
    st->stats[kQac] = st->gd_cur + rem[0] * ((double)a.nx * a.ny * a.nz);
    if (mode == 2) {
      const double ntot = (double)a.nx * a.ny * a.nz;
      st->stats[kQac] = gd[2];  // the starting state's, from the spectral z pass
      st->stats[1] = st->mean_kh[12] + 0.5 * gd[1] / ntot;
      for (int c = 0; c < 6; ++c) {
        st->stats[2 + c] = st->mean_kh[c];
        st->stats[8 + c] = st->mean_kh[6 + c];
      }
      st->st.iters = 1;
      st->st.residual = 0.0;
      st->st.done = 1;
    }
    st->gd_cur = gd[0];
    return;
  }
  if (mode == 1) return;
  if (part == 1) {
    double sm[kQac];
    sum_partials<kQac>(a.part_ac + (size_t)inst * nblk_x * kQac, nblk_x, sm, scratch);
    if (threadIdx.x != 0) return;
    // on the spectral path stress, strain and elastic energy come from part 0
    for (int q = 0; q < kQac; ++q)
      if (mode != 2 || q == 0 || q >= 14) st->stats[q] = sm[q];
    return;
  }
  if (part == 2) {
    double bad[kQres];
    sum_partials<kQres>(a.part_res + (size_t)inst * nblk_x * kQres, nblk_x, bad, scratch);
    if (threadIdx.x == 0 && bad[0] > 0.0) st->st.nonfinite = 1;
    return;
  }
  __shared__ float mm[2];
  const float* pm = a.part_mm + 2 * (size_t)inst * nblk_x;
  float mn = 3.0e38f, mx = -3.0e38f;
#pragma unroll 4
  for (int b = threadIdx.x; b < nblk_x; b += blockDim.x) {
    mn = fminf(mn, pm[2 * b]);
    mx = fmaxf(mx, pm[2 * b + 1]);
  }
  block_minmax(mn, mx, mm);
  if (threadIdx.x != 0) return;
  st->stats[kQac + 1] = mm[0];
  st->stats[kQac + 2] = mm[1];
}

// Homogeneous spectral path after its forward x pass: the step's load and
// status, <f_a> from the FP64 sums of the pass; the mean strain from the
// mixed condition, <sigma>_S = sigma_bar_S with <eps>_E = eps_bar_E and
// <sigma> = C : (<eps> - sum_a <f_a> eps0_a); the mean elastic force
// <sigma> : eps0_a (added to the xi = 0 coefficient by the z pass) and the
// mean-field part of the elastic energy.
__device__ inline void kh_begin_mean(const KArgs& a, int inst, int nblk, double* scratch) {
  double s[kQac];
  sum_partials<kQac>(a.part_ac + (size_t)inst * nblk * kQac, nblk, s, scratch);
  if (threadIdx.x != 0) return;
  DevState* st = a.state + inst;
  const double* ld = a.loads + 12 * (size_t)inst;
  for (int c = 0; c < 6; ++c) {
    st->eps_target[c] = ld[c];
    st->sig_target[c] = ld[6 + c];
  }
  st->st.done = 0;
  st->st.iters = 0;
  const double* kd = a.khd + (size_t)inst * kKhdStride;
  const double ntot = (double)a.nx * a.ny * a.nz;
  // every array below is indexed by constants only (fully unrolled loops),
  // so it stays in registers
  double es[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int r = 0; r < kMaxVar; ++r) {
    if (r >= a.nv) break;
    const double fr = s[14 + r] / ntot;
#pragma unroll
    for (int c = 0; c < 6; ++c) es[c] += fr * kd[72 + 6 * r + c];
  }
  double d[6], rs[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) d[c] = ((a.stress_mask >> c) & 1u) ? 0.0 : ld[c] - es[c];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double acc = ld[6 + i];
#pragma unroll
    for (int j = 0; j < 6; ++j) acc -= kd[6 * i + j] * d[j];
    rs[i] = acc;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i)
    if ((a.stress_mask >> i) & 1u) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < 6; ++j)
        if ((a.stress_mask >> j) & 1u) acc += kd[36 + 6 * i + j] * rs[j];
      d[i] = acc;
    }
  double sg[6], e2 = 0.0;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) acc += kd[6 * i + j] * d[j];
    sg[i] = acc;
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    st->mean_kh[c] = ntot * sg[c];
    st->mean_kh[6 + c] = ntot * (d[c] + es[c]);
    e2 += (c < 3 ? 1.0 : 2.0) * sg[c] * d[c];
  }
  st->mean_kh[12] = 0.5 * ntot * e2;
  for (int q = 0; q < a.nv; ++q) {
    double work = 0.0;
    for (int c = 0; c < 6; ++c) work += (c < 3 ? 1.0 : 2.0) * sg[c] * kd[72 + 6 * q + c];
    st->kh_drive[q] = (double)a.LDt * ntot * work;
  }
}

// Macro-step residual: max over the instance's blocks.
__device__ inline void resid_fin(const KArgs& a, int inst, int nblk) {
  __shared__ float mm[2];
  const float* pm = a.part_mm + 2 * (size_t)inst * nblk;
  float mx = 0.f;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) mx = fmaxf(mx, pm[2 * b + 1]);
  block_minmax(0.f, mx, mm);
  if (threadIdx.x == 0) a.state[inst].resid_max = mm[1];
}

// One-block-per-instance finalize kernels. (Folding them into the last
// block of the x passes needs a device-scope fence in every block, which on
// this multi-L2 part writes back the L2 and costs far more than a launch.)
// Convergence test of every instance (skipped for converged ones), then the
// instance's status published: seq counts the launches, and with a.pub the
// whole Status goes to host-visible memory, seq last after a system-scope
// fence, so the host can wait on seq instead of copying and synchronising.
__global__ __launch_bounds__(1024) void k_fin_res(const KArgs a, int nblk) {
  __shared__ double scratch[1024];
  DevState* st = a.state + blockIdx.x;
  if (!st->st.done) fin_res(a, blockIdx.x, nblk, scratch);
  if (threadIdx.x != 0) return;
  const int seq = st->st.seq + 1;
  st->st.seq = seq;
  if (a.pub) {
    Status* dst = a.pub + blockIdx.x;
    dst->residual = st->st.residual;
    dst->iters = st->st.iters;
    dst->done = st->st.done;
    dst->nonfinite = st->st.nonfinite;
    dst->ready = st->st.ready;
    dst->pf_change = st->st.pf_change;
    dst->pf_iters = st->st.pf_iters;
    __threadfence_system();
    __hip_atomic_store(&dst->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

__global__ __launch_bounds__(1024) void k_fin_ac(const KArgs a, int nblk_x, int nblk_z, int mode) {
  __shared__ double scratch[1024];
  if (a.guard_ready && !a.state[0].st.ready) return;
  fin_ac(a, blockIdx.x, nblk_x, nblk_z, mode, blockIdx.y, scratch);
}


__global__ __launch_bounds__(1024) void k_resid_fin(const KArgs a, int nblk) { resid_fin(a, blockIdx.x, nblk); }

// Fixed point over the update: max change of solve number it over the
// instance's blocks.
__global__ __launch_bounds__(1024) void k_fin_pc(const KArgs a, int nblk, int it) {
  __shared__ float mm[2];
  const float* pm = a.part_pc + 2 * (size_t)blockIdx.x * nblk;
  float mx = 0.f;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) mx = fmaxf(mx, pm[2 * b + 1]);
  block_minmax(0.f, mx, mm);
  if (threadIdx.x == 0) {
    a.state[blockIdx.x].st.pf_change = mm[1];
    a.state[blockIdx.x].st.pf_iters = it;
  }
}

// Largest grain id of a field (checked against the grain count at set-up):
// block maxima of a grid-stride pass, reduced on the host.
__global__ __launch_bounds__(256) void k_gid_max(const uint8_t* __restrict__ gid, size_t n, int* __restrict__ out) {
  __shared__ int red[256];
  int m = 0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    m = max(m, (int)gid[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

}  // namespace pft

// ====================================================================== host
namespace pfl {
using namespace pft;

bool supported_axis(int n) {
  return n == 32 || n == 48 || n == 64 || n == 96 || n == 128 || n == 192 || n == 256 || n == 384 ||
         n == 512;
}

template <int M>
static int rows_per_block_t() { return xthreads<M>() / (M / XPlan<M>::E); }

int rows_per_block(int nx) {
  switch (nx / 2) {
    case 16: return rows_per_block_t<16>();
    case 24: return rows_per_block_t<24>();
    case 32: return rows_per_block_t<32>();
    case 48: return rows_per_block_t<48>();
    case 64: return rows_per_block_t<64>();
    case 96: return rows_per_block_t<96>();
    case 128: return rows_per_block_t<128>();
    case 192: return rows_per_block_t<192>();
    case 256: return rows_per_block_t<256>();
  }
  return 0;
}

// x-pass blocks per instance (the rows of one block never straddle two
// instances: every supported ny * nz is a multiple of the rows per block).
static int x_blocks_inst(const KArgs& a) {
  const int r = rows_per_block(a.nx);
  return (a.nz * a.ny + r - 1) / r;
}

int x_blocks(const KArgs& a) { return a.ninst * x_blocks_inst(a); }

// z-pass partial blocks per instance, for the widest use (the Allen-Cahn
// pass over ncomp variants, or the spectral path's narrower tiles).
static int z_blocks_inst(const KArgs& a, int ncomp) {
  const int ac = z_tiles_x(a, kColTile) * a.ny * ncomp;
  const int kh = z_tiles_inst(a, 8);
  return ac > kh ? ac : kh;
}

int z_blocks(const KArgs& a, int ncomp) { return a.ninst * z_blocks_inst(a, ncomp); }


#define PF_SWITCH_M(nx, BODY)                \
  switch ((nx) / 2) {                         \
    case 16: { constexpr int M = 16; BODY; } break;  \
    case 24: { constexpr int M = 24; BODY; } break;  \
    case 32: { constexpr int M = 32; BODY; } break;  \
    case 48: { constexpr int M = 48; BODY; } break;  \
    case 64: { constexpr int M = 64; BODY; } break;  \
    case 96: { constexpr int M = 96; BODY; } break;  \
    case 128: { constexpr int M = 128; BODY; } break; \
    case 192: { constexpr int M = 192; BODY; } break; \
    case 256: { constexpr int M = 256; BODY; } break; \
    default: return hipErrorInvalidValue;     \
  }

#define PF_SWITCH_N(n, BODY)                 \
  switch (n) {                                \
    case 32: { constexpr int N = 32; BODY; } break;   \
    case 48: { constexpr int N = 48; BODY; } break;   \
    case 64: { constexpr int N = 64; BODY; } break;   \
    case 96: { constexpr int N = 96; BODY; } break;   \
    case 128: { constexpr int N = 128; BODY; } break; \
    case 192: { constexpr int N = 192; BODY; } break; \
    case 256: { constexpr int N = 256; BODY; } break; \
    case 384: { constexpr int N = 384; BODY; } break; \
    case 512: { constexpr int N = 512; BODY; } break; \
    default: return hipErrorInvalidValue;     \
  }

hipError_t group_ready(const KArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_group_ready, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t strain_mean(const KArgs& a, const float* field, int inst, hipStream_t s) {
  hipLaunchKernelGGL(k_strain_mean, dim3(6), dim3(1024), 0, s, a, field, inst);
  return hipGetLastError();
}

hipError_t step_begin(const KArgs& a, hipStream_t st) {
  k_step_begin<<<(a.ninst + 63) / 64, 64, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t ms_x_forward(const KArgs& a, hipStream_t s) {
  switch (a.nv) {
    case 1: return ms_x_forward_v1(a, s);
    case 2: return ms_x_forward_v2(a, s);
    case 3: return ms_x_forward_v3(a, s);
    case 4: return ms_x_forward_v4(a, s);
    case 5: return ms_x_forward_v5(a, s);
    case 6: return ms_x_forward_v6(a, s);
  }
  return hipErrorInvalidValue;
}


// ---------------------------------------------------- plans of y/z passes
template <int N, int K>
static int radices_of(int* elems, int (&r)[8]) {
  using RI = RadixInfo<typename PV<N, K>::R>;
  *elems = PV<N, K>::E;
  for (int i = 0; i < RI::n; ++i) r[i] = RI::r[i];
  return RI::n;
}

template <int N>
static int radices_n(int k, int* elems, int (&r)[8]) {
  switch (k) {
    case 0: return radices_of<N, 0>(elems, r);
    case 1: return radices_of<N, 1>(elems, r);
    case 2: return radices_of<N, 2>(elems, r);
  }
  return 0;
}

int plan_radices(int n, int k, int* elems, int (&radices)[8]) {
  *elems = 0;
  switch (n) {
    case 32: return radices_n<32>(k, elems, radices);
    case 48: return radices_n<48>(k, elems, radices);
    case 64: return radices_n<64>(k, elems, radices);
    case 96: return radices_n<96>(k, elems, radices);
    case 128: return radices_n<128>(k, elems, radices);
    case 192: return radices_n<192>(k, elems, radices);
    case 256: return radices_n<256>(k, elems, radices);
    case 384: return radices_n<384>(k, elems, radices);
    case 512: return radices_n<512>(k, elems, radices);
  }
  return 0;
}

bool plan_fits(int pass, int n, int k, int tile) {
  int e = 0, r[8];
  if (plan_radices(n, k, &e, r) == 0) return false;
  const int kmax = (pass == 1 || pass == 3) ? 1 : 2;
  const bool tile_ok = pass == 2 ? tile == kColTile : (tile == 8 || tile == 16);
  return k <= kmax && tile_ok && tile * (n / e) <= 1024;
}

// A column kernel is instantiated only for the plans and tiles whose block
// fits (the launchers below return hipErrorInvalidValue otherwise).
template <int N, int DIR, int C, int K>
static hipError_t y_launch(const KArgs& a, int ncomp, hipStream_t s) {
  if constexpr (col_threads<N, K, C>() <= 1024) {
    if (a.nz % C) return hipErrorInvalidValue;  // a plane block's z lie in one instance
    const dim3 grid(z_tiles_x(a, C), a.nz * a.ninst, ncomp);
    k_y<N, DIR, C, K><<<grid, dim3(col_threads<N, K, C>()), 0, s>>>(a);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int N, int DIR>
static hipError_t y_pass_n(const KArgs& a, int ncomp, hipStream_t s) {
  const bool c8 = a.ytile == 8;
  switch (a.yplan) {
    case 0: return c8 ? y_launch<N, DIR, 8, 0>(a, ncomp, s) : y_launch<N, DIR, 16, 0>(a, ncomp, s);
    case 1: return c8 ? y_launch<N, DIR, 8, 1>(a, ncomp, s) : y_launch<N, DIR, 16, 1>(a, ncomp, s);
    case 2: return c8 ? y_launch<N, DIR, 8, 2>(a, ncomp, s) : y_launch<N, DIR, 16, 2>(a, ncomp, s);
  }
  return hipErrorInvalidValue;
}

hipError_t y_pass(const KArgs& a, int ncomp, int dir, hipStream_t s) {
  if (dir > 0) {
    PF_SWITCH_N(a.ny, return (y_pass_n<N, 1>(a, ncomp, s)));
  } else {
    PF_SWITCH_N(a.ny, return (y_pass_n<N, -1>(a, ncomp, s)));
  }
  return hipErrorInvalidValue;
}

hipError_t ms_finalize_residual(const KArgs& a, hipStream_t s) {
  k_fin_res<<<a.ninst, 1024, 0, s>>>(a, x_blocks_inst(a));
  return hipGetLastError();
}


template <int N, int C, int K>
static hipError_t zms_launch(const KArgs& a, hipStream_t s) {
  if constexpr (K <= 1 && col_threads<N, K, C>() <= 1024) {
    const dim3 grid(z_tiles_inst(a, C) * a.ninst);
    k_z_ms<N, C, K><<<grid, dim3(col_threads<N, K, C>()), 0, s>>>(a, x_blocks_inst(a));
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int N>
static hipError_t ms_z_green_n(const KArgs& a, hipStream_t s) {
  const bool c16 = a.ztile_ms == 16;
  switch (a.zplan_ms) {
    case 0: return c16 ? zms_launch<N, 16, 0>(a, s) : zms_launch<N, 8, 0>(a, s);
    case 1: return c16 ? zms_launch<N, 16, 1>(a, s) : zms_launch<N, 8, 1>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t ms_z_green(const KArgs& a, hipStream_t s) {
  PF_SWITCH_N(a.nz, return ms_z_green_n<N>(a, s));
  return hipErrorInvalidValue;
}

hipError_t ms_x_inverse(const KArgs& a, hipStream_t s) {
  const dim3 grid(x_blocks(a));
  PF_SWITCH_M(a.nx, (k_x_inv_ms<M><<<grid, xthreads<M>(), 0, s>>>(a)));
  return hipGetLastError();
}


hipError_t ac_x_forward(const KArgs& a, hipStream_t s) {
  switch (a.nv) {
    case 1: return ac_x_forward_v1(a, s);
    case 2: return ac_x_forward_v2(a, s);
    case 3: return ac_x_forward_v3(a, s);
    case 4: return ac_x_forward_v4(a, s);
    case 5: return ac_x_forward_v5(a, s);
    case 6: return ac_x_forward_v6(a, s);
  }
  return hipErrorInvalidValue;
}

template <int N, bool GK, bool WG, int K>
static hipError_t zac_launch(const KArgs& a, int mode, hipStream_t s) {
  if constexpr (col_threads<N, K, kColTile>() <= 1024) {
    const dim3 grid(z_tiles_x(a, kColTile), a.ny * a.ninst, a.nv);
    k_z_ac<N, GK, WG, K><<<grid, dim3(col_threads<N, K, kColTile>()), 0, s>>>(a, mode);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int N, bool GK, bool WG>
static hipError_t ac_z_k(const KArgs& a, int mode, hipStream_t s) {
  switch (a.zplan_ac) {
    case 0: return zac_launch<N, GK, WG, 0>(a, mode, s);
    case 1: return zac_launch<N, GK, WG, 1>(a, mode, s);
    case 2: return zac_launch<N, GK, WG, 2>(a, mode, s);
  }
  return hipErrorInvalidValue;
}

template <int N>
static hipError_t ac_z_n(const KArgs& a, int mode, hipStream_t s) {
  const bool wg = mode == 2 || a.lapf != nullptr;
  if (a.gk && wg) return ac_z_k<N, true, true>(a, mode, s);
  if (a.gk) return ac_z_k<N, true, false>(a, mode, s);
  if (wg) return ac_z_k<N, false, true>(a, mode, s);
  return ac_z_k<N, false, false>(a, mode, s);
}

hipError_t ac_z_update(const KArgs& a, int mode, hipStream_t s) {
  PF_SWITCH_N(a.nz, return ac_z_n<N>(a, mode, s));
  return hipErrorInvalidValue;
}

hipError_t ac_x_inverse(const KArgs& a, hipStream_t s) {
  const dim3 grid(x_blocks(a));
  PF_SWITCH_M(a.nx, (k_x_inv_ac<M><<<grid, xthreads<M>(), 0, s>>>(a)));
  return hipGetLastError();
}

hipError_t pc_x_forward(const KArgs& a, hipStream_t s) {
  switch (a.nv) {
    case 1: return pc_x_forward_v1(a, s);
    case 2: return pc_x_forward_v2(a, s);
    case 3: return pc_x_forward_v3(a, s);
    case 4: return pc_x_forward_v4(a, s);
    case 5: return pc_x_forward_v5(a, s);
    case 6: return pc_x_forward_v6(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t pc_finalize(const KArgs& a, int it, hipStream_t s) {
  k_fin_pc<<<a.ninst, 1024, 0, s>>>(a, x_blocks_inst(a), it);
  return hipGetLastError();
}

hipError_t ac_finalize(const KArgs& a, int mode, hipStream_t s) {
  k_fin_ac<<<dim3(a.ninst, mode == 1 ? 1 : 4), 1024, 0, s>>>(a, x_blocks_inst(a), z_partials_inst(a, mode), mode);
  return hipGetLastError();
}

hipError_t kh_x_forward(const KArgs& a, int resid, hipStream_t s) {
  switch (a.nv) {
    case 1: return kh_x_forward_v1(a, resid, s);
    case 2: return kh_x_forward_v2(a, resid, s);
    case 3: return kh_x_forward_v3(a, resid, s);
  }
  return hipErrorInvalidValue;
}

hipError_t ct_x_forward(const KArgs& a, const float* prev, int n_steps, hipStream_t s) {
  switch (a.nv) {
    case 1: return ct_x_forward_v1(a, prev, n_steps, s);
    case 2: return ct_x_forward_v2(a, prev, n_steps, s);
    case 3: return ct_x_forward_v3(a, prev, n_steps, s);
  }
  return hipErrorInvalidValue;
}

hipError_t kh_residual(const KArgs& a, const float* prev, int n_steps, hipStream_t s) {
  const dim3 grid(x_blocks(a));
  PF_SWITCH_M(a.nx, (k_x_resid<M><<<grid, xthreads<M>(), 0, s>>>(a, prev, (float)n_steps)));
  k_resid_fin<<<a.ninst, 1024, 0, s>>>(a, x_blocks_inst(a));
  return hipGetLastError();
}


template <int N, bool GK, int V, int C, int K>
static hipError_t kh_z_nk(const KArgs& a, int mode, hipStream_t s) {
  if constexpr (K <= 1 && col_threads<N, K, C>() <= 1024) {
    const dim3 grid(z_tiles_inst(a, C) * a.ninst);
    k_z_kh<N, V, GK, C, K><<<grid, dim3(col_threads<N, K, C>()), 0, s>>>(a, mode, x_blocks_inst(a));
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <bool GK, int V, int C, int K>
static hipError_t kh_z_launch(const KArgs& a, int mode, hipStream_t s) {
  PF_SWITCH_N(a.nz, return (kh_z_nk<N, GK, V, C, K>(a, mode, s)));
  return hipErrorInvalidValue;
}

template <bool GK, int V>
static hipError_t kh_z_tile(const KArgs& a, int mode, hipStream_t s) {
  const bool c8 = kh_tile_of(a) == 8;
  switch (a.zplan_kh) {
    case 0: return c8 ? kh_z_launch<GK, V, 8, 0>(a, mode, s) : kh_z_launch<GK, V, 16, 0>(a, mode, s);
    case 1: return c8 ? kh_z_launch<GK, V, 8, 1>(a, mode, s) : kh_z_launch<GK, V, 16, 1>(a, mode, s);
  }
  return hipErrorInvalidValue;
}

template <bool GK>
hipError_t kh_z_update_t(const KArgs& a, int mode, hipStream_t s) {
  switch (a.nv) {
    case 1: return kh_z_tile<GK, 1>(a, mode, s);
    case 2: return kh_z_tile<GK, 2>(a, mode, s);
    case 3: return kh_z_tile<GK, 3>(a, mode, s);
  }
  return hipErrorInvalidValue;
}

hipError_t kh_z_update(const KArgs& a, int mode, hipStream_t s) {
  return a.gk ? kh_z_update_t<true>(a, mode, s) : kh_z_update_t<false>(a, mode, s);
}

hipError_t raw_x_forward(const KArgs& a, const float* real, int ncomp, hipStream_t s) {
  const dim3 grid(x_blocks(a), ncomp);
  PF_SWITCH_M(a.nx, (k_x_fwd_raw<M><<<grid, xthreads<M>(), 0, s>>>(a, real)));
  return hipGetLastError();
}

template <int N, int DIR, int K>
static hipError_t zraw_launch(const KArgs& a, int ncomp, hipStream_t s) {
  if constexpr (col_threads<N, K, kColTile>() <= 1024) {
    const dim3 grid(z_tiles_x(a, kColTile), a.ny * a.ninst, ncomp);
    k_z_raw<N, DIR, K><<<grid, dim3(col_threads<N, K, kColTile>()), 0, s>>>(a);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int N, int DIR>
static hipError_t raw_z_n(const KArgs& a, int ncomp, hipStream_t s) {
  switch (a.zplan_ac) {
    case 0: return zraw_launch<N, DIR, 0>(a, ncomp, s);
    case 1: return zraw_launch<N, DIR, 1>(a, ncomp, s);
    case 2: return zraw_launch<N, DIR, 2>(a, ncomp, s);
  }
  return hipErrorInvalidValue;
}

hipError_t raw_z(const KArgs& a, int ncomp, int dir, hipStream_t s) {
  if (dir > 0) {
    PF_SWITCH_N(a.nz, return (raw_z_n<N, 1>(a, ncomp, s)));
  } else {
    PF_SWITCH_N(a.nz, return (raw_z_n<N, -1>(a, ncomp, s)));
  }
  return hipErrorInvalidValue;
}

template <int N, int K, bool DIV>
static hipError_t gd_launch(const KArgs& a, hipStream_t s) {
  if constexpr (col_threads<N, K, kColTile>() <= 1024) {
    const dim3 grid(z_tiles_x(a, kColTile), a.ny * a.ninst);
    if constexpr (DIV)
      k_z_div<N, K><<<grid, dim3(col_threads<N, K, kColTile>()), 0, s>>>(a);
    else
      k_z_grad<N, K><<<grid, dim3(col_threads<N, K, kColTile>()), 0, s>>>(a);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int N, bool DIV>
static hipError_t gd_n(const KArgs& a, hipStream_t s) {
  switch (a.zplan_ac) {
    case 0: return gd_launch<N, 0, DIV>(a, s);
    case 1: return gd_launch<N, 1, DIV>(a, s);
    case 2: return gd_launch<N, 2, DIV>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t grad_z(const KArgs& a, hipStream_t s) {
  PF_SWITCH_N(a.nz, return (gd_n<N, false>(a, s)));
  return hipErrorInvalidValue;
}

hipError_t div_z(const KArgs& a, hipStream_t s) {
  PF_SWITCH_N(a.nz, return (gd_n<N, true>(a, s)));
  return hipErrorInvalidValue;
}

hipError_t flux_x(const KArgs& a, hipStream_t s) {
  const dim3 grid(x_blocks(a));
  PF_SWITCH_M(a.nx, (k_x_flux<M><<<grid, xthreads<M>(), 0, s>>>(a)));
  return hipGetLastError();
}

hipError_t grain_id_max(const uint8_t* gid, size_t n, int* out, int nblk, hipStream_t s) {
  k_gid_max<<<nblk, 256, 0, s>>>(gid, n, out);
  return hipGetLastError();
}

hipError_t raw_x_inverse(const KArgs& a, float* real, int ncomp, float scale, hipStream_t s) {
  const dim3 grid(x_blocks(a), ncomp);
  PF_SWITCH_M(a.nx, (k_x_inv_raw<M><<<grid, xthreads<M>(), 0, s>>>(a, real, scale)));
  return hipGetLastError();
}

}  // namespace pfl
