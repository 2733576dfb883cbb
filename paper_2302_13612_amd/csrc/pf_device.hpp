// Shared declarations between the HIP kernels and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pft {

constexpr int kMaxVar = 6;
constexpr int kColTile = 16;       // spectral columns per y/z block
constexpr int kZmsTile = 8;        // default columns per block of the Green z pass

// Quantities reduced per block (FP64 partial sums / extrema).
constexpr int kQms = 6;                 // sum of stress (mixed condition)
constexpr int kQres = 2;                // |eps_new - eps_old|^2, |eps_new|^2
constexpr int kQac = 2 + 6 + 6 + kMaxVar;  // G_dw, G_me, sum sigma, sum eps, sum eta
constexpr int kQgd = 3;                 // Parseval gradient sum (new state), spectral elastic
                                        // energy, gradient sum of the starting state (spectral path)

// Status copied back to the host after each fixed-point iteration.
struct Status {
  double residual;
  int32_t iters;
  int32_t done;
  int32_t nonfinite;
  int32_t ready;      // instance 0 of a group: every instance converged (guarded update)
  double pf_change;   // max |f^i - f^{i-1}| of the last solve of the update's fixed point
  int32_t pf_iters;   // solves of that fixed point in the last step
  int32_t seq;        // status publications of the fixed point (one per k_fin_res launch)
};

// Device-resident state of a context (FP64 scalars).
struct DevState {
  double ebar_cur[6];    // mean strain of the current iterate
  double ebar_field[6];  // mean strain of the strain field in memory
  double ebar_next[6];   // mean strain for the next iterate
  double ebar_h[4][6];   // mean strains of the last four converged fields (latest first)
  double ebar_base[6];   // mean of the field the current iterate is formed from
  double eps_target[6];  // load: prescribed mean strain
  double sig_target[6];  // load: prescribed mean stress
  double gd_cur;         // gradient energy sum of the current order parameter
  double stats[32];      // reductions of the last step (layout in the host)
  double mean_kh[13];    // homogeneous spectral path: N<sigma> (6), N<eps> (6),
                         // mean-field elastic energy sum (1)
  double kh_drive[kMaxVar];  // L dt N <sigma> : eps0_a (mean of the elastic force)
  double resid_max;          // max |residual| of the last macro-step check
  Status st;
};

// Per-instance reference medium: packed C0 (21) then its compliance S0 (36,
// Voigt stress -> tensor-Voigt strain).
constexpr int kRefStride = 21 + 36;


// Per-instance tables of the homogeneous spectral path (one stiffness C in
// the whole instance, linear h, no plastic strain). Float part: C packed (21),
// sigma0_a = C : eps0_a (6 per variant), W_ab = eps0_a : C : eps0_b (V x V).
// Double part: M = C in tensor-Voigt form (36), the inverse of its
// stress-controlled block embedded in 6x6 (36), eps0_a (6 per variant).
constexpr int kKhStride = 21 + 6 * kMaxVar + kMaxVar * kMaxVar;
constexpr int kKhdStride = 36 + 36 + 6 * kMaxVar;
// anisotropic gradient energy, per instance and variant: 6 coefficients of
// the semi-implicit denominator 1 + sum D k k and 6 of the energy symbol
// sum G k k over integer wave numbers (xx yy zz, then doubled yz xz xy)
constexpr int kGkStride = 12 * kMaxVar;
constexpr int kKhMaxVar = 3;       // variants handled by the spectral path (2 V <= 6 spectra)

// Everything a kernel needs, passed by value. A context holds ninst
// independent instances of one grid size stacked along z: fields are
// [comp][inst][z][y][x] and spectra [comp][inst][z][y][sh]; every x-pass block
// and every z column lies in one instance.
struct KArgs {
  int nx, ny, nz, nh, nv;     // grid of one instance, nh = nx/2+1, number of variants
  int ninst;                  // instances stacked along z
  int sh;                     // spectral row stride (complex elements, >= ncol)
  int ncol;                   // columns of a spectral row: nx/2, the Nyquist coefficient
                              // kx = nx/2 being kept in a plane of its own (nqo), or nh
                              // when it stays in the row (nq_row: the caller's layout)
  int nq_row;                 // 1: Nyquist coefficient at column nx/2 of its row
  size_t cs;                  // stride between spectral components (complex elements)
  size_t nqo;                 // offset of the Nyquist plane [inst][z][y] in a component
  int h_kind;
  int n_grains, tab_stride;
  float A, LDt;               // double-well height, L*dt
  float ax, ay, az;           // 2 L dt kappa (2 pi / (n dx))^2 per axis
  double gx, gy, gz;          // (2 pi / (n dx))^2 per axis (energy)
  float inv_ntot;
  double tol;
  const float* ref;           // [ninst][kRefStride] reference medium per instance
  const double* bss;          // [ninst][36] mixed-condition correction matrix
  const double* loads;        // [ninst][12] prescribed mean strain (6) and stress (6)
  int tab_inst;               // table stride between instances (n_grains * tab_stride)
  const float* kh;            // [ninst][kKhStride] or null
  const double* khd;          // [ninst][kKhdStride] or null
  const float* gk;            // [ninst][kGkStride] or null (isotropic kappa)
  const float* mob;           // [nz][ny][nx] relative mobility, or null (uniform)
  float* lapf;                // [nv][nz][ny][nx] 2 div(K grad f) of the state (with mob)
  const float* krem;          // [n_grains][nv][6] K_a^g - kbar_a I (tensor-Voigt): per-grain
                              // gradient tensors (the explicit remainder), or null
  double* part_rem;           // [x blocks] sums of grad f . (K - kbar I) . grad f, with krem
  float cdx, cdy, cdz;        // 2 pi / (n dx) per axis (first derivatives)
  float gscale;               // 2 kappa (isotropic symbol) or 2 (tables carry K)
  float* pf_base;             // [nv][nz][ny][nx] f^n + L dt m mech of the step, kept for
                              // the fixed point over the update, or null (one solve)
  float* part_pc;             // per-block (0, max |f^i - f^{i-1}|) of that fixed point
  uint32_t stress_mask;
  // fields
  float* eta;                 // [nv][ninst][nz][ny][nx]
  float* eps;                 // [6][ninst][nz][ny][nx] strain the iterate is formed from
  float* eps_out;             // where the inverse pass writes the new iterate; with
                              // iter_mode != 0 the forward pass first stores the
                              // extrapolated iterate there (the inverse pass's old value)
  const float* eps_h1;        // converged strain of the step before (iter_mode >= 1)
  const float* eps_h2;        // of the one before that (iter_mode >= 2)
  const float* eps_h3;        // and of the one before that (iter_mode 3)
  int iter_mode;              // first iterate of a step: 0 eps, 1 linear extrapolation
                              // 2 eps - h1, 2 quadratic 3 (eps - h1) + h2, 3 cubic
                              // 4 eps - 6 h1 + 4 h2 - h3
  float* sig;                 // [6][ninst][nz][ny][nx] (only written on request)
  const float* epsp;          // [6][ninst][nz][ny][nx] or null
  const uint8_t* gid;         // [nz][ny][nx] or null (one instance only)
  const float* tables;        // [ninst][n_grains][tab_stride]
  const float* rot;           // [n_grains][12] crystal->sample rotations (row-major 3x3), or null
  float xtab[21 + 27 * kMaxVar];  // crystal-frame table shared by every grain (rotation form)
  float2* spec;               // [6][ninst][nz][ny][sh]
  const float2* tw_xh;        // length nx/2
  const float2* tw_x;         // length nx
  const float2* tw_y;         // length ny
  const float2* tw_z;         // length nz
  double* part_ms;            // per-block partials
  double* part_res;
  double* part_ac;
  float* part_mm;             // per-block min/max of eta
  double* part_gd;
  DevState* state;            // [ninst]
  int save_stress;
  int skip_done;              // y pass: skip instances whose fixed point has converged
  int ytile;                  // columns per block of the y passes (8 or 16; 0: 16)
  int ztile_kh;               // columns per block of the spectral path's z pass (8 or 16;
                              // 0: 16 for one variant, else 8)
  int yplan;                  // FFT plan variant of the y passes (0, 1, 2)
  int ztile_ms, zplan_ms;     // Green z pass: columns per block (0: 8) and plan variant (0, 1)
  int zplan_ac;               // Allen-Cahn z pass: plan variant (0, 1, 2)
  int zplan_kh;               // spectral path's z pass: plan variant (0, 1)
  Status* pub;                // [ninst] host-visible copy of each instance's Status, or null:
                              // the fixed point's finalize writes it there for the host to poll
  int guard_ready;            // update passes: run only if state[0].st.ready (a step
                              // replayed as a graph, its fixed point done on the device)
};

// Nyquist coefficient (kx = nx/2) of spectral row `row` (counted over all
// instances) of component c.
__host__ __device__ inline float2* nyq_at(const KArgs& a, int c, size_t row) {
  return a.spec + c * a.cs + (a.nq_row ? row * a.sh + a.nx / 2 : a.nqo + row);
}

// Packed upper-triangle index of a symmetric 6x6 matrix.
__host__ __device__ constexpr int sym6(int i, int j) {
  return i <= j ? i * 6 - i * (i - 1) / 2 + (j - i) : j * 6 - j * (j - 1) / 2 + (i - j);
}

}  // namespace pft

// Launchers implemented in pf_kernels.hip. Each returns a hipError_t value.
namespace pfl {
using pft::KArgs;
int rows_per_block(int nx);
int x_blocks(const KArgs& a);
int z_blocks(const KArgs& a, int ncomp);
hipError_t step_begin(const KArgs& a, hipStream_t s);
// state[0].st.ready = every instance of the group converged
hipError_t group_ready(const KArgs& a, hipStream_t s);
// mean of each component of instance inst of a strain field -> its
// DevState::ebar_field (after the caller replaced the strain)
hipError_t strain_mean(const KArgs& a, const float* field, int inst, hipStream_t s);
hipError_t ms_x_forward(const KArgs& a, hipStream_t s);
hipError_t y_pass(const KArgs& a, int ncomp, int dir, hipStream_t s);
hipError_t ms_z_green(const KArgs& a, hipStream_t s);
hipError_t ms_x_inverse(const KArgs& a, hipStream_t s);
hipError_t ac_x_forward(const KArgs& a, hipStream_t s);
// mode 0 update, 1 energy only, 2 gradient force 2 div(K grad f) in place
hipError_t ac_z_update(const KArgs& a, int mode, hipStream_t s);
hipError_t ac_x_inverse(const KArgs& a, hipStream_t s);
// Fixed point over the update: the right-hand side of a further solve from
// the kept base and the chemical force of the latest iterate, R2C in x; and
// the per-instance max change of a solve into Status (solve number it).
hipError_t pc_x_forward(const KArgs& a, hipStream_t s);
hipError_t pc_finalize(const KArgs& a, int it, hipStream_t s);
hipError_t ms_finalize_residual(const KArgs& a, hipStream_t s);
hipError_t ac_finalize(const KArgs& a, int mode, hipStream_t s);  // 0 step, 1 init, 2 spectral path
// 0 update, 1 L dt dF/df; the block owning xi = 0 of an instance first takes
// the step's load and the mean fields (kh_begin_mean)
hipError_t kh_z_update(const KArgs& a, int mode, hipStream_t s);
hipError_t raw_x_forward(const KArgs& a, const float* real, int ncomp, hipStream_t s);
hipError_t raw_z(const KArgs& a, int ncomp, int dir, hipStream_t s);
hipError_t raw_x_inverse(const KArgs& a, float* real, int ncomp, float scale, hipStream_t s);
// block maxima (nblk of them, into out) of n grain ids
hipError_t grain_id_max(const uint8_t* gid, size_t n, int* out, int nblk, hipStream_t s);
bool supported_axis(int n);
// FFT plans of the y and z passes: elements per thread and radix stages of
// variant k on an axis of length n (0 stages if there is no such plan), and
// whether a pass of that plan and column tile fits one block.
int plan_radices(int n, int k, int* elems, int (&radices)[8]);
// pass: 0 y passes (k 0..2, tile 8/16), 1 Green z pass (k 0..1, tile 8/16),
// 2 Allen-Cahn z pass (k 0..2, tile 16), 3 spectral z pass (k 0..1, tile 8/16)
bool plan_fits(int pass, int n, int k, int tile);
// per variant count, one translation unit each
hipError_t ms_x_forward_v1(const KArgs& a, hipStream_t s);
hipError_t ms_x_forward_v2(const KArgs& a, hipStream_t s);
hipError_t ms_x_forward_v3(const KArgs& a, hipStream_t s);
hipError_t ms_x_forward_v4(const KArgs& a, hipStream_t s);
hipError_t ms_x_forward_v5(const KArgs& a, hipStream_t s);
hipError_t ms_x_forward_v6(const KArgs& a, hipStream_t s);
hipError_t ac_x_forward_v1(const KArgs& a, hipStream_t s);
hipError_t ac_x_forward_v2(const KArgs& a, hipStream_t s);
hipError_t ac_x_forward_v3(const KArgs& a, hipStream_t s);
hipError_t ac_x_forward_v4(const KArgs& a, hipStream_t s);
hipError_t ac_x_forward_v5(const KArgs& a, hipStream_t s);
hipError_t ac_x_forward_v6(const KArgs& a, hipStream_t s);
hipError_t pc_x_forward_v1(const KArgs& a, hipStream_t s);
hipError_t pc_x_forward_v2(const KArgs& a, hipStream_t s);
hipError_t pc_x_forward_v3(const KArgs& a, hipStream_t s);
hipError_t pc_x_forward_v4(const KArgs& a, hipStream_t s);
hipError_t pc_x_forward_v5(const KArgs& a, hipStream_t s);
hipError_t pc_x_forward_v6(const KArgs& a, hipStream_t s);
hipError_t kh_x_forward_v1(const KArgs& a, int resid, hipStream_t s);
hipError_t kh_x_forward_v2(const KArgs& a, int resid, hipStream_t s);
hipError_t kh_x_forward_v3(const KArgs& a, int resid, hipStream_t s);
// resid = 1: the transforms of f and L dt chem(f), for kh_z_update(mode 1)
hipError_t kh_x_forward(const KArgs& a, int resid, hipStream_t s);
hipError_t ct_x_forward_v1(const KArgs& a, const float* prev, int n_steps, hipStream_t s);
hipError_t ct_x_forward_v2(const KArgs& a, const float* prev, int n_steps, hipStream_t s);
hipError_t ct_x_forward_v3(const KArgs& a, const float* prev, int n_steps, hipStream_t s);
// Forward x pass of the residual of a macro step of n_steps plain steps from
// prev to the current order parameter: 3V spectral components (see k_x_fwd_ct)
hipError_t ct_x_forward(const KArgs& a, const float* prev, int n_steps, hipStream_t s);
// Residual of that macro step, inverse pass: r = f~ - prev + n_steps g, g the
// output of ct_x_forward, y forward (3V), kh_z_update(mode 2), y inverse (V):
// per-instance max |r| into DevState::resid_max.
hipError_t kh_residual(const KArgs& a, const float* prev, int n_steps, hipStream_t s);
// The explicit remainder of per-grain gradient tensors, 2 div((K(x) - kbar I)
// grad f) of the order parameters: grad_z and flux_x (with the remainder's
// gradient energy into a.part_rem) around raw x and y transforms on the
// components V .. 4V-1, then div_z adds L dt times the divergence to the
// update's y-transformed right-hand side (components 0 .. V-1).
hipError_t grad_z(const KArgs& a, hipStream_t s);
hipError_t flux_x(const KArgs& a, hipStream_t s);
hipError_t div_z(const KArgs& a, hipStream_t s);
}  // namespace pfl
